// Host-side launchers of the FFT pass kernels (implemented in nm_passes.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nm {

// Spectral constants of the operator and of the reference-medium preconditioner.
struct SpecParams {
    double L1, L2, L3;
    int n1, n2, n3;
    int dim;          // 2 (plane strain, n3 == 1, z components held at zero) or 3
    double inv_ntot;  // 1 / (n1 n2 n3): normalization of one forward/inverse round trip
    double bdt2;      // beta dt^2
    double rhobar;    // volume-averaged density
    double Cbar[21];  // volume-averaged Voigt stiffness (upper triangle, row major)
};

// Fused stage in front of the x-direction real-to-complex transform.
enum XFwdMode { XF_PLAIN = 0, XF_PUPDATE = 1, XF_UPDATE = 2 };
// Fused stage after the x-direction complex-to-real transform.
enum XInvMode { XI_PLAIN = 0, XI_OPERATOR = 1, XI_PRECOND = 2 };
// Pointwise operator applied between the forward and inverse z transforms.
enum ZOp { ZOP_GRAD = 0, ZOP_DIV = 1, ZOP_PRECOND = 2 };

// Device scalar block shared by the Krylov kernels (all double).
enum ScalarSlot { S_ALPHA = 0, S_BETA = 1, S_FIRST = 2, S_RZ = 3, S_PQ = 4, S_RR = 5, S_COUNT = 8 };

struct XFwdArgs {
    const void* src;      // XF_PLAIN: input field; XF_PUPDATE: z
    void* p;              // XF_PUPDATE: p (in/out); XF_UPDATE: p (in)
    void* x;              // XF_UPDATE: x (in/out)
    void* r;              // XF_UPDATE: r (in/out)
    const void* q;        // XF_UPDATE: q (in)
    const double* scal;   // device scalars
    double* partials;     // XF_UPDATE: per-block partial sums of r.r
    void* spec;           // output half spectrum
    long nlines;          // number of x lines (components x n2 x n3)
};

struct XInvArgs {
    const void* spec;     // input half spectrum
    void* out;            // output real field
    const void* aux;      // XI_OPERATOR: p ; XI_PRECOND: r
    const uint16_t* phase;
    const void* rho;      // per-phase density (T)
    const uint8_t* mask;  // Gamma voxel mask or null
    double* partials;     // per-block partial dot products or null
    long nlines;
    long lines_per_comp;  // n2 * n3
    int dim;
};

// Number of blocks a launch uses (sizes the partials array).
int xfwd_blocks(int n1, long nlines);
int xinv_blocks(int n1, long nlines);

template <typename T> int launch_xfwd(int mode, int n1, const XFwdArgs& a, const void* tw, hipStream_t s);
template <typename T> int launch_xinv(int mode, int n1, const XInvArgs& a, const void* tw, hipStream_t s);
// In-place x-inverse, Voigt stress sigma = C_g : eps, x-forward on 6 components.
template <typename T>
int launch_xstress(int n1, void* spec, long lines_per_comp, long NS, const uint16_t* phase, const void* C21,
                   const void* tw, hipStream_t s);
// In-place transform of ncomp components along y (dir -1 forward, +1 inverse).
template <typename T>
int launch_ypass(int dir, int n1, int n2, int n3, int ncomp, long NS, void* spec, const void* tw, hipStream_t s);
// In-place z-forward, pointwise operator, z-inverse.
template <typename T>
int launch_zspec(int op, const SpecParams& sp, long NS, void* spec, const void* tw, hipStream_t s);

} // namespace nm
