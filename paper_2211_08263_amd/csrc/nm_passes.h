// Host-side launchers of the FFT pass kernels (implemented in nm_passes.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nm {

// Spectral constants of the operator and of the reference-medium preconditioner.
struct SpecParams {
    double L1, L2, L3;
    double k1, k2, k3; // 2 pi / L_i
    int n1, n2, n3;
    int dim;          // 2 (plane strain, n3 == 1, z components held at zero) or 3
    double inv_ntot;  // 1 / (n1 n2 n3): normalization of one forward/inverse round trip
    double inv_n1, inv_n2, inv_n3;
    double bdt2;      // beta dt^2
    double rhobar;    // volume-averaged density
    double Cbar[21];  // volume-averaged Voigt stiffness (upper triangle, row major)
    const double* stop = nullptr; // device flag: when non-zero, kernels given this struct exit at once
    // Finite-difference differentiation rules: device table of the frequency each bin's
    // derivative uses in place of the spectral xi (n1 + n2 + n3 entries, axis after axis, indexed
    // by bin), or null for the spectral derivative.
    const double* mfreq = nullptr;
    // Several independent fields at once (multi-right-hand-side solves): bk fields whose
    // spectra lie bs elements apart; the column passes take the field from blockIdx.z.
    long bs = 0;
    int bk = 1;
};


// Layout of a half-spectrum buffer: element (c, kz, ky, kx) at
// c * cs + kz * ps + ky * M + kx.  The plane and component strides may carry
// padding so that the strided z pass does not hit power-of-two strides.
struct SpecLayout {
    int M;          // n1 / 2
    int n2, n3;
    int log2n2;
    long ps;        // kz (plane) stride, >= n2 * M
    long cs;        // component stride, >= n3 * ps
    const double* stop = nullptr; // device flag: when non-zero, kernels given this layout exit at once
    // Several fields at once: nb fields of bc components each, bs elements apart (bc == 0: one
    // field, components cs apart).
    int nb = 1;
    int bc = 0;
    long bs = 0;
    __host__ __device__ __forceinline__ long comp(long c) const { return bc ? (c / bc) * bs + (c % bc) * cs : c * cs; }
    __host__ __device__ __forceinline__ long line(long l) const
    {
        // x line l = (component, kz, ky) in row-major order
        const long yz = l % ((long)n2 * n3), c = l / ((long)n2 * n3);
        return comp(c) + (yz >> log2n2) * ps + (yz & (n2 - 1)) * (long)M;
    }
};

// Fused stage in front of the x-direction real-to-complex transform.
// XF_UPDATE: r -= alpha q with the partial sums of r.r (the direction update is fused into
// the preconditioner's last pass instead, launch_xpupdate).
// XF_EXPLICIT: the displacement update u <- u + dt v + dt^2/2 a of the central-difference
// scheme (written back to u) before the transform.
enum XFwdMode { XF_PLAIN = 0, XF_UPDATE = 2, XF_EXPLICIT = 3 };
// Fused stage after the x-direction complex-to-real transform.
// XI_EXPLICIT: with o = (dt/2) div sigma from the transform, v <- v + dt/2 a + o/rho and
// a <- 2 o / (dt rho) (central-difference velocity before the Gamma force; eq.
// Explicit_linear_momentum_arranged_3D).
enum XInvMode { XI_PLAIN = 0, XI_OPERATOR = 1, XI_PRECOND = 2, XI_EXPLICIT = 3 };
// Axis-wise derivative stages of the operator on x-spectral (kx, y, z) data:
//   YOP_DERIV : S[3+j] = D_y S[j], j < 3
//   ZOP_STRAIN: S2 = Voigt strain (eps11, eps22, eps33, g23, g13, g12) / n1 from
//               U = S[0..2] and D_y U = S[3..5] (D_x = i xi1, D_z by a z round trip)
//   YOP_DIV   : S[0..2] = (i xi1 s11 + D_y s12, i xi1 s12 + D_y s22, i xi1 s13 + D_y s23), sigma in S2
//   ZOP_DIVZ  : S[j] = -beta dt^2 / n1 (S[j] + D_z sigma_j3)
enum ColOp { YOP_DERIV = 0, YOP_DIV = 1, ZOP_STRAIN = 2, ZOP_DIVZ = 3 };

// Device scalar block shared by the Krylov kernels (all double).
// S_STOP .. S_MODE drive a Krylov loop that runs several iterations between host checks:
// the residual reduction counts iterations (S_ITER) and raises S_STOP once r.r <= S_THR2
// (S_MODE 0) or the count reaches S_LIMIT; every guarded kernel after that returns at once.
enum ScalarSlot {
    S_ALPHA = 0, S_BETA = 1, S_FIRST = 2, S_RZ = 3, S_PQ = 4, S_RR = 5,
    S_STOP = 8, S_ITER = 9, S_THR2 = 10, S_LIMIT = 11, S_MODE = 12, S_COUNT = 16
};

struct XFwdArgs {
    const void* src;      // XF_PLAIN: input field
    void* u = nullptr;        // XF_EXPLICIT: displacement (in/out)
    const void* v = nullptr;  // XF_EXPLICIT: velocity
    const void* a = nullptr;  // XF_EXPLICIT: acceleration
    double dt = 0.0;          // XF_EXPLICIT: time increment
    void* r;              // XF_UPDATE: r (in/out)
    const void* q;        // XF_UPDATE: q (in)
    const double* scal;   // device scalars
    double* partials;     // XF_UPDATE: per-block partial sums of r.r
    void* spec;           // output half spectrum
    SpecLayout lay;
    long nlines;          // number of x lines (components x n2 x n3)
    long lines_per_batch = 0; // several fields: x lines per field (their device scalars lie S_COUNT apart)
};

struct XInvArgs {
    const void* spec;     // input half spectrum
    SpecLayout lay;
    void* out;            // output real field
    const void* aux;      // XI_OPERATOR: p ; XI_PRECOND: r
    const uint16_t* phase;
    const void* rho;      // per-phase density (T)
    const uint8_t* mask;  // Gamma voxel mask or null
    double* partials;     // per-block partial dot products or null
    long nlines;
    long lines_per_comp;  // n2 * n3
    int dim;
    void* p = nullptr;            // launch_xpupdate: search direction (in/out); XI_EXPLICIT: velocity (in/out)
    void* x = nullptr;            // launch_xpupdate: iterate (in/out); XI_EXPLICIT: acceleration (in/out)
    double dt = 0.0;              // XI_EXPLICIT: time increment
    const double* scal = nullptr; // launch_xpupdate: device scalars (alpha, beta, first)
    long lines_per_batch = 0;     // several fields: x lines per field (their scalars lie S_COUNT apart)
};

// Number of blocks a launch uses (sizes the partials array).
int xfwd_blocks(int n1, long nlines);
int xinv_blocks(int n1, long nlines);

template <typename T> int launch_xfwd(int mode, int n1, const XFwdArgs& a, const void* tw, hipStream_t s);
template <typename T> int launch_xinv(int mode, int n1, const XInvArgs& a, const void* tw, hipStream_t s);
// In place on the half spectrum a.spec: z = mask(x-inverse), p = z + beta p with the
// deferred x += alpha p_old (p = z while scal[S_FIRST] is set), spectrum <- x-forward(p).
template <typename T> int launch_xpupdate(int n1, const XInvArgs& a, const void* tw, hipStream_t s);
// In-place x-inverse, Voigt stress sigma = C_g : eps, x-forward on 6 components.
template <typename T>
int launch_xstress(int n1, void* spec, const SpecLayout& lay, const uint16_t* phase, const void* C21, const void* tw,
                   hipStream_t s);
// In-place transform of ncomp components along y (dir -1 forward, +1 inverse).
template <typename T>
int launch_ypass(int dir, int ncomp, const SpecLayout& lay, void* spec, const void* tw, hipStream_t s);
// (the y pass reads lay.stop)
// Axis-wise derivative stages of the operator (ColOp); S and S2 are two 6-component spectra.
template <typename T>
int launch_colop(int op, const SpecParams& sp, const SpecLayout& lay, void* S, void* S2, const void* tw,
                 hipStream_t s);
// Preconditioner z pass in place: z-forward, (beta dt^2 K + rhobar I)^-1, z-inverse.
// partials (or null): per-block sums of r . z taken on the spectrum (Parseval), one per
// block of zprecond_blocks<T>(sp).
template <typename T>
int launch_zprecond(const SpecParams& sp, const SpecLayout& lay, void* spec, const void* tw, hipStream_t s,
                    double* partials = nullptr);
template <typename T> int zprecond_blocks(const SpecParams& sp);

} // namespace nm
