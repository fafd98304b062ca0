// FFT pass kernels of the operator of eq. (Fourier_ND_A) and of the
// reference-medium preconditioner of eqs. (precond)-(acous), for gfx950.
//
// Data layout.  Real fields are SoA [component][z][y][x] with x fastest.
// Half spectra are [component][kz][ky][kx] complex with kx in [0, n1/2):
// slot kx = 0 holds X(0) + i X(n1/2) (both real after the x transform).
// Because the discrete frequency of the Nyquist bin is taken as zero, the
// kx = 0 and kx = n1/2 planes see the same multiplier, every multiplier is
// Hermitian in (ky, kz), and the packed slot goes through the y/z passes
// and the pointwise operators unchanged.  Forward transforms are
// unnormalized, inverse ones too; 1/(n1 n2 n3) is folded into the spectral
// multipliers.
//
// Passes of one operator apply q = A p (7 kernels; the derivatives are taken
// axis by axis, D_x as i xi1 on x spectra, D_y and D_z by single-axis round
// trips, and every pointwise stage is fused into a transform pass):
//   x-fwd (3) | y: U -> D_y U (3 -> 6) | z: strain (6 -> 6) |
//   x-inv, sigma = C : eps, x-fwd (6) | y: D_y and i xi1 terms of div (5 -> 3) |
//   z: D_z terms, -beta dt^2 scale (6 -> 3) | x-inv + rho p (3).
// The preconditioner z = M r is x-fwd | y-fwd | z-fwd, (beta dt^2 K + rhobar I)^-1,
// z-inv | y-inv | x-inv (3 components throughout).  Inside PCG its x-inv is fused with
// the direction update and the x-fwd of the next operator apply (k_xpupdate), and the
// residual update r -= alpha q rides on the preconditioner's x-fwd (XF_UPDATE).
#include "nm_common.h"
#include "nm_fft.h"
#include "nm_passes.h"

// Strain components whose loads the stress pass keeps in flight ahead of its transforms
// (FP64 holds fewer: its registers limit the occupancy).
#ifndef NM_STRESS_PF64
#define NM_STRESS_PF64 2
#endif
// The stress pass keeps its twiddles in registers across its twelve transforms (measured at
// 256^3: 6% faster in FP64; in FP32, 132 -> 136 VGPRs at the same occupancy, 1-2% faster with
// the streaming accesses below, 5% slower before them).
#ifndef NM_STRESS_TWREG64
#define NM_STRESS_TWREG64 1
#endif
#ifndef NM_STRESS_TWREG32
#define NM_STRESS_TWREG32 1
#endif
// Column passes address their tiles as a uniform base plus 32-bit lane offsets.
#ifndef NM_COL_OFF32
#define NM_COL_OFF32 1
#endif
#ifndef NM_STRESS_PF32
#define NM_STRESS_PF32 6
#endif
// FP64 stress pass on 512-long x lines: one strain component's loads in flight instead of two
// (measured at 512^3: 4.34 -> 3.17 ms; twiddles from LDS instead of registers 3.38 ms, radix 8
// 4.07 ms)
#ifndef NM_STRESS512_TWREG64
#define NM_STRESS512_TWREG64 NM_STRESS_TWREG64
#endif
#ifndef NM_STRESS512_PF64
#define NM_STRESS512_PF64 1
#endif
#ifndef NM_STRESS512_R64
#define NM_STRESS512_R64 NM_STRESS_R64
#endif
// Nontemporal (streaming) loads (bit 0) and stores (bit 1) of the spectra and fields that a
// pass reads or writes once, per pass family and precision.  Measured at 256^3 (500 grains):
// FP64 operator 1.72 -> 1.63 ms, preconditioner 0.91 -> 0.84 ms, Newmark step 40.7 -> 38.0 ms;
// the FP32 passes gain less and lose where the preconditioner's column passes stream their
// loads (0.43 -> 0.48 ms), so FP32 streams only the x passes and the column operators' stores
// (mixed-precision step 24.3 -> 23.2 ms).
#ifndef NM_STRESS_NT64
#define NM_STRESS_NT64 3
#endif
#ifndef NM_STRESS_NT32
#define NM_STRESS_NT32 3
#endif
#ifndef NM_XFWD_NT64
#define NM_XFWD_NT64 3
#endif
#ifndef NM_XFWD_NT32
#define NM_XFWD_NT32 3
#endif
#ifndef NM_XINV_NT64
#define NM_XINV_NT64 3
#endif
#ifndef NM_XINV_NT32
#define NM_XINV_NT32 3
#endif
#ifndef NM_XPUP_NT64
#define NM_XPUP_NT64 3
#endif
#ifndef NM_XPUP_NT32
#define NM_XPUP_NT32 3
#endif
#ifndef NM_YPASS_NT64
#define NM_YPASS_NT64 2
#endif
#ifndef NM_YPASS_NT32
#define NM_YPASS_NT32 0
#endif
#ifndef NM_COLOP_NT64
#define NM_COLOP_NT64 3
#endif
#ifndef NM_COLOP_NT32
#define NM_COLOP_NT32 2
#endif
#ifndef NM_ZPRE_NT64
#define NM_ZPRE_NT64 2
#endif
#ifndef NM_ZPRE_NT32
#define NM_ZPRE_NT32 0
#endif
#define NM_NT(FAM, T) (sizeof(T) == 8 ? NM_##FAM##_NT64 : NM_##FAM##_NT32)
// FP32 x passes: a line group past the last line reads line 0 instead of skipping its loads, so
// the loads carry no branch (measured: FP32 stress pass 214 -> 206 us at 256^3; the same in FP64
// costs 30%, so FP64 keeps the guarded loads).
#define NM_TAIL_LOADS(T) (sizeof(T) == 4)
// per column operator (ColOp 0..3), defaulting to the family's setting.  The FP32 strain pass
// (ZOP_STRAIN) streams its loads as well: 170 -> 151 us at 256^3, FP32 operator 0.856 -> 0.838 ms
// (the same pass's setting moves the FP64 stress pass after it by up to 20 us either way, and the
// FP64 operator by no more than the noise, so FP64 keeps the family setting).
#ifndef NM_COLOP2_NT32
#define NM_COLOP2_NT32 3
#endif
#ifndef NM_COLOP0_NT64
#define NM_COLOP0_NT64 NM_COLOP_NT64
#endif
#ifndef NM_COLOP0_NT32
#define NM_COLOP0_NT32 NM_COLOP_NT32
#endif
#ifndef NM_COLOP1_NT64
#define NM_COLOP1_NT64 NM_COLOP_NT64
#endif
#ifndef NM_COLOP1_NT32
#define NM_COLOP1_NT32 NM_COLOP_NT32
#endif
#ifndef NM_COLOP2_NT64
#define NM_COLOP2_NT64 NM_COLOP_NT64
#endif
#ifndef NM_COLOP2_NT32
#define NM_COLOP2_NT32 NM_COLOP_NT32
#endif
#ifndef NM_COLOP3_NT64
#define NM_COLOP3_NT64 NM_COLOP_NT64
#endif
#ifndef NM_COLOP3_NT32
#define NM_COLOP3_NT32 NM_COLOP_NT32
#endif
#define NM_COLOP_OP_NT(OP, T)                                                                                          \
    ((OP) == 0   ? (sizeof(T) == 8 ? NM_COLOP0_NT64 : NM_COLOP0_NT32)                                                     \
     : (OP) == 1 ? (sizeof(T) == 8 ? NM_COLOP1_NT64 : NM_COLOP1_NT32)                                                     \
     : (OP) == 2 ? (sizeof(T) == 8 ? NM_COLOP2_NT64 : NM_COLOP2_NT32)                                                     \
                 : (sizeof(T) == 8 ? NM_COLOP3_NT64 : NM_COLOP3_NT32))

namespace nm {

// Early exit of a guarded kernel once the Krylov loop has stopped (uniform branch).
__device__ __forceinline__ bool stopped(const double* stop) { return stop && *stop != 0.0; }

// ---------------------------------------------------------------------------
// Deterministic reductions (fixed shuffle tree per wave, fixed order across waves)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block sum for 256-thread blocks, valid in thread 0.
__device__ __forceinline__ double block_sum256(double v)
{
    __shared__ double sh[kBlock / 64];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < kBlock / 64; i++) s += sh[i];
    }
    return s;
}

// R2C post-processing: from Z = FFT_M(x[2n] + i x[2n+1]) to the packed
// half spectrum X(k), k < M, with X(0) + i X(M) in slot 0.  zk = Z[k],
// zm = Z[(M-k) mod M], wk = exp(-2 pi i k / N1).
template <typename V> __device__ __forceinline__ V r2c_post(int k, V zk, V zm, V wk)
{
    using S = decltype(zk.x);
    if (k == 0) return V{zk.x + zk.y, zk.x - zk.y};
    V zc = conjv(zm);
    V e = cscale(cadd(zk, zc), (S)0.5);
    V d = csub(zk, zc);
    V o = V{(S)0.5 * d.y, (S)-0.5 * d.x}; // (zk - conj zm) / (2 i)
    return cadd(e, cmul(wk, o));
}

// C2R pre-processing: Z[k] = (X[k] + conj X[M-k]) + i w^k (X[k] - conj X[M-k]),
// w = exp(+2 pi i / N1); slot 0 carries X(0) + i X(M).
template <typename V> __device__ __forceinline__ V c2r_pre(int k, V xk, V xm, V wk_fwd)
{
    if (k == 0) return V{xk.x + xk.y, xk.x - xk.y};
    V xc = conjv(xm);
    V a = cadd(xk, xc);
    V b = csub(xk, xc);
    V wb = cmul(conjv(wk_fwd), b);
    return V{a.x - wb.y, a.y + wb.x};
}

// Copy the twiddle table of length L into LDS (block-cooperative; the caller
// synchronizes the block before use).
template <int L, typename V> __device__ __forceinline__ void stage_twiddles(V* dst, const V* __restrict__ tw)
{
    if constexpr (L >= 2) {
        for (int i = threadIdx.x; i < L; i += blockDim.x) dst[i] = tw[tw_offset(L) + i];
    }
}

// ---------------------------------------------------------------------------
// x direction: real lines of N1 points, M = N1/2 complex points per line
// ---------------------------------------------------------------------------
template <typename T, int N1, int R, int MODE>
__global__ __launch_bounds__(kBlock) void k_xfwd(XFwdArgs a, const cx_t<T>* __restrict__ tw)
{
    if (stopped(a.lay.stop)) return;
    using V = cx_t<T>;
    constexpr int M = N1 / 2, G = M / R, LPB = kBlock / G, LP = M;
    static_assert(G <= 64, "an x line must live inside one wavefront");
    __shared__ V lds[LPB * LP];
    __shared__ V twsm[M + N1];
    stage_twiddles<M>(twsm, tw);
    stage_twiddles<N1>(twsm + M, tw);
    __syncthreads();
    const V* twM = twsm;
    const V* twN = twsm + M;
    const int tid = threadIdx.x, ll = tid / G, t = tid % G;
    const long line = (long)blockIdx.x * LPB + ll;
    const bool valid = line < a.nlines;
    const long off = line * M;
    V v[R];
    double part = 0.0;
#pragma unroll
    for (int m = 0; m < R; m++) v[m] = V{0, 0};
    if (valid) {
        if constexpr (MODE == XF_PLAIN) {
            const V* src = (const V*)a.src + off;
#pragma unroll
            for (int m = 0; m < R; m++) v[m] = ld_nt<NM_NT(XFWD, T)>(src + t + m * G);
        } else if constexpr (MODE == XF_EXPLICIT) {
            // u_n = u_{n-1} + dt v_{n-1} + dt^2/2 a_{n-1}   (eq. Central_diff_rule)
            const T dt = (T)a.dt, h2 = (T)(0.5 * a.dt * a.dt);
            V* u = (V*)a.u + off;
            const V* vv = (const V*)a.v + off;
            const V* aa = (const V*)a.a + off;
#pragma unroll
            for (int m = 0; m < R; m++) {
                const int i = t + m * G;
                const V uo = ld_nt<NM_NT(XFWD, T)>(u + i), vo = ld_nt<NM_NT(XFWD, T)>(vv + i),
                        ao = ld_nt<NM_NT(XFWD, T)>(aa + i);
                const V un = V{uo.x + dt * vo.x + h2 * ao.x, uo.y + dt * vo.y + h2 * ao.y};
                st_nt<NM_NT(XFWD, T)>(u + i, un);
                v[m] = un;
            }
        } else {
            // r -= alpha q and the partial sums of r.r
            const T alpha = (T)a.scal[(a.lines_per_batch ? line / a.lines_per_batch : 0) * S_COUNT + S_ALPHA];
            V* r = (V*)a.r + off;
            const V* q = (const V*)a.q + off;
#pragma unroll
            for (int m = 0; m < R; m++) {
                const int i = t + m * G;
                V qq = ld_nt<NM_NT(XFWD, T)>(q + i), rr = ld_nt<NM_NT(XFWD, T)>(r + i);
                rr = V{rr.x - alpha * qq.x, rr.y - alpha * qq.y};
                st_nt<NM_NT(XFWD, T)>(r + i, rr);
                part += (double)rr.x * (double)rr.x + (double)rr.y * (double)rr.y;
                v[m] = rr;
            }
        }
    }
    LineAddr<R, (int)sizeof(V)> addr{ll * LP};
    group_fft<M, R, -1, true>(v, t, lds, addr, twM);
#pragma unroll
    for (int m = 0; m < R; m++) lds[addr(t + m * G)] = v[m];
    group_sync<true>();
    V mir[R];
#pragma unroll
    for (int m = 0; m < R; m++) mir[m] = lds[addr((M - (t + m * G)) & (M - 1))];
    if (valid) {
        V* out = (V*)a.spec + a.lay.line(line);
#pragma unroll
        for (int m = 0; m < R; m++) {
            const int k = t + m * G;
            st_nt<NM_NT(XFWD, T)>(out + k, r2c_post(k, v[m], mir[m], twN[k]));
        }
    }
    if constexpr (MODE == XF_UPDATE) {
        double s = block_sum256(part);
        if (threadIdx.x == 0) a.partials[blockIdx.x] = s;
    }
}

template <typename T, int N1, int R, int MODE>
__global__ __launch_bounds__(kBlock) void k_xinv(XInvArgs a, const cx_t<T>* __restrict__ tw)
{
    if (stopped(a.lay.stop)) return;
    using V = cx_t<T>;
    constexpr int M = N1 / 2, G = M / R, LPB = kBlock / G, LP = M;
    static_assert(G <= 64, "an x line must live inside one wavefront");
    __shared__ V lds[LPB * LP];
    __shared__ V twsm[M + N1];
    stage_twiddles<M>(twsm, tw);
    stage_twiddles<N1>(twsm + M, tw);
    __syncthreads();
    const V* twM = twsm;
    const V* twN = twsm + M;
    const int tid = threadIdx.x, ll = tid / G, t = tid % G;
    const long line = (long)blockIdx.x * LPB + ll;
    const bool valid = line < a.nlines;
    const bool ld_ok = NM_TAIL_LOADS(T) || valid;
    const long lineA = NM_TAIL_LOADS(T) && !valid ? 0 : line;
    const long off = lineA * M;
    V v[R];
    const long soff = a.lay.line(lineA);
#pragma unroll
    for (int m = 0; m < R; m++) v[m] = ld_ok ? ld_nt<NM_NT(XINV, T)>((const V*)a.spec + soff + t + m * G) : V{0, 0};
    // the real-space operands of the fused stage are fetched before the transform
    V au[R];
    uint32_t ph[R];
    uint16_t mk[R];
    const long vline = lineA % a.lines_per_comp;
    V ao[R];
    if constexpr (MODE == XI_EXPLICIT) {
        const V* vp = (const V*)a.p + off;
        const V* ap = (const V*)a.x + off;
#pragma unroll
        for (int m = 0; m < R; m++) {
            const int n = t + m * G;
            au[m] = ld_ok ? ld_nt<NM_NT(XINV, T)>(vp + n) : V{0, 0};
            ao[m] = ld_ok ? ld_nt<NM_NT(XINV, T)>(ap + n) : V{0, 0};
            ph[m] = ld_ok ? ((const uint32_t*)a.phase)[vline * M + n] : 0u;
            mk[m] = 0;
        }
    } else if constexpr (MODE != XI_PLAIN) {
        const V* aux = (const V*)a.aux + off;
#pragma unroll
        for (int m = 0; m < R; m++) {
            const int n = t + m * G;
            au[m] = (ld_ok && a.aux) ? ld_nt<NM_NT(XINV, T)>(aux + n) : V{0, 0};
            ph[m] = (ld_ok && MODE == XI_OPERATOR) ? ((const uint32_t*)a.phase)[vline * M + n] : 0u;
            mk[m] = (ld_ok && a.mask) ? ((const uint16_t*)a.mask)[vline * M + n] : (uint16_t)0;
        }
    }
    LineAddr<R, (int)sizeof(V)> addr{ll * LP};
#pragma unroll
    for (int m = 0; m < R; m++) lds[addr(t + m * G)] = v[m];
    group_sync<true>();
#pragma unroll
    for (int m = 0; m < R; m++) {
        const int k = t + m * G;
        V xm = lds[addr((M - k) & (M - 1))];
        v[m] = c2r_pre(k, v[m], xm, twN[k]);
    }
    group_sync<true>();
    group_fft<M, R, +1, true>(v, t, lds, addr, twM);
    double part = 0.0;
    if (valid) {
        V* out = (V*)a.out + off;
        if constexpr (MODE == XI_PLAIN) {
#pragma unroll
            for (int m = 0; m < R; m++) st_nt<NM_NT(XINV, T)>(out + t + m * G, v[m]);
        } else if constexpr (MODE == XI_EXPLICIT) {
            // o = dt/2 div sigma: v <- v + dt/2 a + o / rho, a <- (2/dt) o / rho
            const bool zero_comp = (a.dim == 2) && ((line / a.lines_per_comp) % 3 == 2);
            const T* rho = (const T*)a.rho;
            const T hdt = (T)(0.5 * a.dt), idt2 = (T)(2.0 / a.dt);
            V* vp = (V*)a.p + off;
            V* ap = (V*)a.x + off;
#pragma unroll
            for (int m = 0; m < R; m++) {
                const int n = t + m * G;
                const T r0 = rho[ph[m] & 0xffffu], r1 = rho[ph[m] >> 16];
                const V o = v[m];
                V vn = V{au[m].x + hdt * ao[m].x + o.x / r0, au[m].y + hdt * ao[m].y + o.y / r1};
                V an = V{idt2 * o.x / r0, idt2 * o.y / r1};
                if (zero_comp) {
                    vn = V{0, 0};
                    an = V{0, 0};
                }
                st_nt<NM_NT(XINV, T)>(vp + n, vn);
                st_nt<NM_NT(XINV, T)>(ap + n, an);
            }
        } else {
            const bool zero_comp = (a.dim == 2) && ((line / a.lines_per_comp) % 3 == 2);
            const T* rho = (const T*)a.rho;
#pragma unroll
            for (int m = 0; m < R; m++) {
                const int n = t + m * G;
                V o = v[m];
                if constexpr (MODE == XI_OPERATOR) {
                    o.x += rho[ph[m] & 0xffffu] * au[m].x;
                    o.y += rho[ph[m] >> 16] * au[m].y;
                }
                if (mk[m] & 0x00ffu) o.x = 0;
                if (mk[m] & 0xff00u) o.y = 0;
                if (zero_comp) o = V{0, 0};
                part += (double)au[m].x * (double)o.x + (double)au[m].y * (double)o.y;
                st_nt<NM_NT(XINV, T)>(out + n, o);
            }
        }
    }
    if constexpr (MODE != XI_PLAIN && MODE != XI_EXPLICIT) {
        double s = block_sum256(part);
        if (threadIdx.x == 0 && a.partials) a.partials[blockIdx.x] = s;
    }
}

// Last pass of the preconditioner fused with the first pass of the next operator apply
// (in place on the half spectrum): z = P x-inv(Z) (the preconditioned residual, masked
// on Gamma), p = z + beta p and the deferred x += alpha p_old (p = z on the first
// iteration), then the x-forward transform of the new p overwrites the line.  The
// preconditioned residual never goes to memory.
template <typename T, int N1, int R>
__global__ __launch_bounds__(kBlock) void k_xpupdate(XInvArgs a, const cx_t<T>* __restrict__ tw)
{
    if (stopped(a.lay.stop)) return;
    using V = cx_t<T>;
    constexpr int M = N1 / 2, G = M / R, LPB = kBlock / G, LP = M;
    static_assert(G <= 64, "an x line must live inside one wavefront");
    __shared__ V lds[LPB * LP];
    __shared__ V twsm[M + N1];
    stage_twiddles<M>(twsm, tw);
    stage_twiddles<N1>(twsm + M, tw);
    __syncthreads();
    const V* twM = twsm;
    const V* twN = twsm + M;
    const int tid = threadIdx.x, ll = tid / G, t = tid % G;
    const long line = (long)blockIdx.x * LPB + ll;
    const bool valid = line < a.nlines;
    const bool ld_ok = NM_TAIL_LOADS(T) || valid;
    const long lineA = NM_TAIL_LOADS(T) && !valid ? 0 : line;
    const long off = lineA * M;
    const long soff = a.lay.line(lineA);
    V* spec = (V*)a.spec;
    V v[R];
#pragma unroll
    for (int m = 0; m < R; m++) v[m] = ld_ok ? ld_nt<NM_NT(XPUP, T)>(spec + soff + t + m * G) : V{0, 0};
    // the real-space operands are fetched before the transforms
    const double* sc = a.scal + ((a.lines_per_batch && valid) ? line / a.lines_per_batch : 0) * S_COUNT;
    const bool first = sc[S_FIRST] != 0.0;
    const T beta = (T)sc[S_BETA];
    const T alpha = (T)sc[S_ALPHA];
    V* p = (V*)a.p + off;
    V* x = (V*)a.x + off;
    V po[R], xo[R];
    uint16_t mk[R];
    const long vline = lineA % a.lines_per_comp;
#pragma unroll
    for (int m = 0; m < R; m++) {
        const int n = t + m * G;
        po[m] = (ld_ok && !first) ? ld_nt<NM_NT(XPUP, T)>(p + n) : V{0, 0};
        xo[m] = (ld_ok && !first) ? ld_nt<NM_NT(XPUP, T)>(x + n) : V{0, 0};
        mk[m] = (ld_ok && a.mask) ? ((const uint16_t*)a.mask)[vline * M + n] : (uint16_t)0;
    }
    LineAddr<R, (int)sizeof(V)> addr{ll * LP};
#pragma unroll
    for (int m = 0; m < R; m++) lds[addr(t + m * G)] = v[m];
    group_sync<true>();
#pragma unroll
    for (int m = 0; m < R; m++) {
        const int k = t + m * G;
        V xm = lds[addr((M - k) & (M - 1))];
        v[m] = c2r_pre(k, v[m], xm, twN[k]);
    }
    group_sync<true>();
    group_fft<M, R, +1, true>(v, t, lds, addr, twM);
    const bool zero_comp = (a.dim == 2) && ((line / a.lines_per_comp) % 3 == 2);
#pragma unroll
    for (int m = 0; m < R; m++) {
        V z = v[m];
        if (mk[m] & 0x00ffu) z.x = 0;
        if (mk[m] & 0xff00u) z.y = 0;
        if (zero_comp) z = V{0, 0};
        if (!first) {
            xo[m] = V{xo[m].x + alpha * po[m].x, xo[m].y + alpha * po[m].y};
            z = V{z.x + beta * po[m].x, z.y + beta * po[m].y};
        }
        v[m] = z;
    }
    if (valid) {
#pragma unroll
        for (int m = 0; m < R; m++) {
            const int n = t + m * G;
            st_nt<NM_NT(XPUP, T)>(p + n, v[m]);
            if (!first) st_nt<NM_NT(XPUP, T)>(x + n, xo[m]);
        }
    }
    group_fft<M, R, -1, true>(v, t, lds, addr, twM);
#pragma unroll
    for (int m = 0; m < R; m++) lds[addr(t + m * G)] = v[m];
    group_sync<true>();
    V mir[R];
#pragma unroll
    for (int m = 0; m < R; m++) mir[m] = lds[addr((M - (t + m * G)) & (M - 1))];
    if (valid) {
#pragma unroll
        for (int m = 0; m < R; m++) {
            const int k = t + m * G;
            st_nt<NM_NT(XPUP, T)>(spec + soff + k, r2c_post(k, v[m], mir[m], twN[k]));
        }
    }
}

// sigma_v = C_v eps_v for one voxel (Voigt, engineering shear; 21 = upper triangle).
template <typename T> __device__ __forceinline__ void voigt_stress(const T* __restrict__ c, const T e[6], T s[6])
{
    // row-major upper triangle offsets: row a starts at a*6 - a*(a-1)/2
    s[0] = c[0] * e[0] + c[1] * e[1] + c[2] * e[2] + c[3] * e[3] + c[4] * e[4] + c[5] * e[5];
    s[1] = c[1] * e[0] + c[6] * e[1] + c[7] * e[2] + c[8] * e[3] + c[9] * e[4] + c[10] * e[5];
    s[2] = c[2] * e[0] + c[7] * e[1] + c[11] * e[2] + c[12] * e[3] + c[13] * e[4] + c[14] * e[5];
    s[3] = c[3] * e[0] + c[8] * e[1] + c[12] * e[2] + c[15] * e[3] + c[16] * e[4] + c[17] * e[5];
    s[4] = c[4] * e[0] + c[9] * e[1] + c[13] * e[2] + c[16] * e[3] + c[18] * e[4] + c[19] * e[5];
    s[5] = c[5] * e[0] + c[10] * e[1] + c[14] * e[2] + c[17] * e[3] + c[19] * e[4] + c[20] * e[5];
}

template <typename T, int N1, int R>
__global__ __launch_bounds__(kBlock) void k_xstress(cx_t<T>* spec, SpecLayout lay, const uint16_t* __restrict__ phase,
                                                    const T* __restrict__ C21, const cx_t<T>* __restrict__ tw)
{
    if (stopped(lay.stop)) return;
    using V = cx_t<T>;
    constexpr int M = N1 / 2, G = M / R, LPB = kBlock / G, LP = M;
    static_assert(G <= 64, "an x line must live inside one wavefront");
    __shared__ V lds[LPB * LP];
    __shared__ V twsm[M + N1];
    stage_twiddles<M>(twsm, tw);
    stage_twiddles<N1>(twsm + M, tw);
    __syncthreads();
    const V* twM = twsm;
    const V* twN = twsm + M;
    const int tid = threadIdx.x, ll = tid / G, t = tid % G;
    const long line = (long)blockIdx.x * LPB + ll;
    const long lpf = (long)lay.n2 * lay.n3; // x lines per component of one field
    const bool valid = line < lpf * lay.nb;
    LineAddr<R, (int)sizeof(V)> addr{ll * LP};
    // the twelve transforms share their twiddles: with TWR they are read once into registers
    constexpr bool TWR = sizeof(T) == 8 ? (N1 == 512 ? NM_STRESS512_TWREG64 : NM_STRESS_TWREG64) : NM_STRESS_TWREG32;
    TwRegs<M, R, V> twr;
    V twn[R];
    if constexpr (TWR) {
        twr.load(t, twM);
#pragma unroll
        for (int m = 0; m < R; m++) twn[m] = twN[t + m * G];
    }
    auto fft_inv = [&](V (&x)[R]) {
        if constexpr (TWR) group_fft_tw<M, R, +1, true>(x, t, lds, addr, twr);
        else group_fft<M, R, +1, true>(x, t, lds, addr, twM);
    };
    auto fft_fwd = [&](V (&x)[R]) {
        if constexpr (TWR) group_fft_tw<M, R, -1, true>(x, t, lds, addr, twr);
        else group_fft<M, R, -1, true>(x, t, lds, addr, twM);
    };
    auto twk = [&](int m, int k) -> V {
        if constexpr (TWR) return twn[m];
        else return twN[k];
    };
    const bool ld_ok = NM_TAIL_LOADS(T) || valid;
    const long lineA = NM_TAIL_LOADS(T) && !valid ? 0 : line;
    const long off = lay.line(lineA), NS = lay.cs;
    // keep the global loads of the next PF strain components in flight while a
    // component is transformed: the fences of the LDS exchanges would otherwise hold
    // each component's loads back until the previous transform is done
    constexpr int PFQ = sizeof(T) == 8 ? (N1 == 512 ? NM_STRESS512_PF64 : NM_STRESS_PF64) : NM_STRESS_PF32;
    constexpr int PF = PFQ < 6 ? PFQ : 6;
    V raw[6][R];
#pragma unroll
    for (int c = 0; c < PF; c++)
#pragma unroll
        for (int m = 0; m < R; m++) raw[c][m] = ld_ok ? ld_nt<NM_NT(STRESS, T)>(spec + c * NS + off + t + m * G) : V{0, 0};
    uint32_t phw[R];
    {
        const uint32_t* ph2 = (const uint32_t*)phase + (valid ? line % lpf : 0) * M;
#pragma unroll
        for (int m = 0; m < R; m++) phw[m] = ph2[t + m * G];
    }
    T e[6][2 * R];
#pragma unroll
    for (int c = 0; c < 6; c++) {
        V v[R];
#pragma unroll
        for (int m = 0; m < R; m++) v[m] = raw[c][m];
        if (c + PF < 6) {
#pragma unroll
            for (int m = 0; m < R; m++) raw[c + PF][m] = ld_ok ? ld_nt<NM_NT(STRESS, T)>(spec + (c + PF) * NS + off + t + m * G) : V{0, 0};
        }
#pragma unroll
        for (int m = 0; m < R; m++) lds[addr(t + m * G)] = v[m];
        group_sync<true>();
#pragma unroll
        for (int m = 0; m < R; m++) {
            const int k = t + m * G;
            v[m] = c2r_pre(k, v[m], lds[addr((M - k) & (M - 1))], twk(m, k));
        }
        group_sync<true>();
        fft_inv(v);
#pragma unroll
        for (int m = 0; m < R; m++) {
            e[c][2 * m] = v[m].x;
            e[c][2 * m + 1] = v[m].y;
        }
    }
    if (valid) {
#pragma unroll
        for (int m = 0; m < R; m++) {
            const uint32_t ph = phw[m];
#pragma unroll
            for (int h = 0; h < 2; h++) {
                const T* cg = C21 + 21 * (h ? (ph >> 16) : (ph & 0xffffu));
                T ee[6], ss[6];
#pragma unroll
                for (int q = 0; q < 6; q++) ee[q] = e[q][2 * m + h];
                voigt_stress(cg, ee, ss);
#pragma unroll
                for (int q = 0; q < 6; q++) e[q][2 * m + h] = ss[q];
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 6; c++) {
        V v[R];
#pragma unroll
        for (int m = 0; m < R; m++) v[m] = V{e[c][2 * m], e[c][2 * m + 1]};
        fft_fwd(v);
#pragma unroll
        for (int m = 0; m < R; m++) lds[addr(t + m * G)] = v[m];
        group_sync<true>();
        V mir[R];
#pragma unroll
        for (int m = 0; m < R; m++) mir[m] = lds[addr((M - (t + m * G)) & (M - 1))];
        group_sync<true>();
        if (valid) {
#pragma unroll
            for (int m = 0; m < R; m++) {
                const int k = t + m * G;
                st_nt<NM_NT(STRESS, T)>(spec + c * NS + off + k, r2c_post(k, v[m], mir[m], twk(m, k)));
            }
        }
    }
}

// ---------------------------------------------------------------------------
// y and z directions: tiles of TX consecutive kx columns, L points each.
// ---------------------------------------------------------------------------
// Column tiles: element p of column c at p * TX + c.  With TX >= 8 complex
// (16-byte elements) each group of 8 consecutive lanes covers all banks, so no
// padding is needed; a compile-time TX (TXC > 0) lets the offsets fold into
// the LDS instructions' immediate fields.  TXC == 0: runtime TX (small grids).
template <int TXC> struct ColAddrT {
    int c, tx;
    __device__ __forceinline__ int operator()(int p) const { return p * (TXC > 0 ? TXC : tx) + c; }
};

template <typename T, int L, int R, int DIR, int BLK, int TXC>
__global__ __launch_bounds__(BLK) void k_ypass(cx_t<T>* __restrict__ data, long colstride, long planestride, long cs,
                                               int TXr, const cx_t<T>* __restrict__ tw, const double* stop, long bs)
{
    if (stopped(stop)) return;
    using V = cx_t<T>;
    constexpr int G = L / R;
    const int TX = TXC > 0 ? TXC : TXr;
    __shared__ V lds[BLK * R]; // TX * L <= BLK R
    __shared__ V twsm[L];
    stage_twiddles<L>(twsm, tw);
    __syncthreads();
    const int tid = threadIdx.x, c = tid % TX, t = tid / TX;
    // component blockIdx.z (of three per field when several fields lie bs apart)
    const long zc = bs ? (long)(blockIdx.z / 3) * bs + (long)(blockIdx.z % 3) * cs : (long)blockIdx.z * cs;
    V* col = data + zc + blockIdx.y * planestride + (long)blockIdx.x * TX + c;
    V v[R];
#pragma unroll
    for (int m = 0; m < R; m++) v[m] = ld_nt<NM_NT(YPASS, T)>(col + (long)(t + m * G) * colstride);
    ColAddrT<TXC> addr{c, TX};
    group_fft<L, R, DIR>(v, t, lds, addr, twsm);
#pragma unroll
    for (int m = 0; m < R; m++) st_nt<NM_NT(YPASS, T)>(col + (long)(t + m * G) * colstride, v[m]);
}

// Frequency of x bin kx (0 <= kx < n1/2; slot 0 also carries the Nyquist bin, zero under every
// rule), of y bin ky and of z bin kz, in the same units as k1 kx.
__device__ __forceinline__ double freq_x(const SpecParams& sp, int kx)
{
    return sp.mfreq ? sp.mfreq[kx] : sp.k1 * kx;
}
__device__ __forceinline__ double freq_y(const SpecParams& sp, int ky)
{
    return sp.mfreq ? sp.mfreq[sp.n1 + ky] : sp.k2 * freq_index(ky, sp.n2);
}
__device__ __forceinline__ double freq_z(const SpecParams& sp, int kz)
{
    return sp.mfreq ? sp.mfreq[sp.n1 + sp.n2 + kz] : sp.k3 * freq_index(kz, sp.n3);
}

// Pointwise operators at frequency (xi1, xi2, xi3).
template <typename T> struct ZOps {
    using V = cx_t<T>;
    // i s (a): multiply by i and a real scale
    static __device__ __forceinline__ V iscale(V a, T s) { return V{-a.y * s, a.x * s}; }
};

// Preconditioner z pass: forward z transforms of the three components, the pointwise
// inverse of beta dt^2 K(xi) + rhobar I (K_ij = Cbar_ikjm xi_k xi_m, eqs. (precond),
// (acous)) scaled by 1 / (n1 n2 n3), inverse z transforms.  Columns of TX kx bins
// at one ky; data in place.
template <typename T, int L, int R, int BLK, int TXC>
__global__ __launch_bounds__(BLK) void k_zprecond(cx_t<T>* __restrict__ data, long NS, long colstride, int TXr,
                                                  SpecParams sp, const cx_t<T>* __restrict__ tw,
                                                  double* __restrict__ partials)
{
    if (stopped(sp.stop)) return;
    using V = cx_t<T>;
    constexpr int G = L / R;
    const int TX = TXC > 0 ? TXC : TXr;
    __shared__ V lds[BLK * R]; // TX * L <= BLK R
    __shared__ V twsm[L > 1 ? L : 2];
    const int tid = threadIdx.x, c = tid % TX, t = tid / TX;
    const int M = sp.n1 / 2;
    const int kx = blockIdx.x * TX + c, ky = blockIdx.y;
    // uniform column-tile base (scalar registers) plus 32-bit per-lane byte offsets
    V* const cb = data + (long)blockIdx.z * sp.bs + (long)ky * M + (long)blockIdx.x * TX;
    const uint32_t lane = (uint32_t)(c * sizeof(V)) + (uint32_t)t * (uint32_t)(colstride * sizeof(V));
    const uint32_t mstep = (uint32_t)(G * colstride * sizeof(V));
    auto at = [&](int j, int m) -> V& { return *(V*)((char*)(cb + j * NS) + (lane + (uint32_t)m * mstep)); };
    // all three components' loads go out before the first transform (the barriers of
    // the LDS exchanges would otherwise hold each load back behind the previous transform)
    auto load3 = [&](V (&v)[3][R]) {
#pragma unroll
        for (int j = 0; j < 3; j++)
#pragma unroll
            for (int m = 0; m < R; m++) v[j][m] = ld_nt<NM_NT(ZPRE, T)>(&at(j, m));
    };
    V u[3][R];
    if constexpr (TXC > 0 && L >= 2 && sizeof(T) == 4) {
        // full FP32 blocks: the twiddle loads go out first and the operands right behind
        // them, so that only the twiddles are waited for before the barrier that publishes
        // them (FP64, at one wave per SIMD, measured faster with the operands loaded after
        // that barrier)
        constexpr int NT = (L + BLK - 1) / BLK;
        V twv[NT];
#pragma unroll
        for (int q = 0; q < NT; q++)
            if (tid + q * BLK < L) twv[q] = tw[tw_offset(L) + tid + q * BLK];
        load3(u);
#pragma unroll
        for (int q = 0; q < NT; q++)
            if (tid + q * BLK < L) twsm[tid + q * BLK] = twv[q];
        __syncthreads();
    } else {
        stage_twiddles<L>(twsm, tw);
        __syncthreads();
        load3(u);
    }
    ColAddrT<TXC> addr{c, TX};
    const V* twL = twsm;
    const T xi1 = (T)freq_x(sp, kx);
    const T bdt2 = (T)sp.bdt2, rb = (T)sp.rhobar, s = (T)sp.inv_ntot;
    // beta dt^2 K(xi) + rhobar I with K = N(xi)^T Cbar N(xi), N the Voigt strain of a plane
    // wave.  At fixed (xi1, xi2) it is quadratic in xi3: N = N12 + xi3 E3 (N12 holds the
    // xi1, xi2 entries, E3 the unit entries that xi3 multiplies), so
    //   beta dt^2 K + rhobar I = A0 + xi3 (A1 + xi3 A2)
    // with A0 = beta dt^2 N12^T C N12 + rhobar I, A1 = beta dt^2 (N12^T C E3 + E3^T C N12),
    // A2 = beta dt^2 E3^T C E3, formed once per thread (symmetric; upper triangles kept).
    auto form = [&](T x1, T x2, T (&A0)[6], T (&A1)[6], T (&A2)[6]) {
        T C[6][6];
        int o = 0;
#pragma unroll
        for (int a = 0; a < 6; a++)
#pragma unroll
            for (int b = a; b < 6; b++) {
                C[a][b] = (T)sp.Cbar[o];
                C[b][a] = (T)sp.Cbar[o];
                o++;
            }
        T CN[6][3], CE[6][3];
#pragma unroll
        for (int a = 0; a < 6; a++) {
            CN[a][0] = C[a][0] * x1 + C[a][5] * x2;
            CN[a][1] = C[a][1] * x2 + C[a][5] * x1;
            CN[a][2] = C[a][3] * x2 + C[a][4] * x1;
            CE[a][0] = C[a][4];
            CE[a][1] = C[a][3];
            CE[a][2] = C[a][2];
        }
        // rows of N12^T X and E3^T X for a 6 x 3 X
        auto n12 = [&](const T (&X)[6][3], int i, int j) -> T {
            return i == 0 ? x1 * X[0][j] + x2 * X[5][j] : i == 1 ? x2 * X[1][j] + x1 * X[5][j] : x2 * X[3][j] + x1 * X[4][j];
        };
        auto e3 = [&](const T (&X)[6][3], int i, int j) -> T { return i == 0 ? X[4][j] : i == 1 ? X[3][j] : X[2][j]; };
        int q = 0;
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = i; j < 3; j++) {
                A0[q] = bdt2 * n12(CN, i, j) + (i == j ? rb : (T)0);
                A1[q] = bdt2 * (n12(CE, i, j) + e3(CN, i, j));
                A2[q] = bdt2 * e3(CE, i, j);
                q++;
            }
    };
#pragma unroll
    for (int j = 0; j < 3; j++) group_fft<L, R, -1>(u[j], t, lds, addr, twL);
    T A0[6], A1[6], A2[6]; // order 00 01 02 11 12 22
    form(xi1, (T)freq_y(sp, ky), A0, A1, A2);
    // per-thread part of r . z in the working precision (24 products at most), summed in
    // FP64 across threads
    T part = 0;
#pragma unroll
    for (int m = 0; m < R; m++) {
        const T x3 = (T)freq_z(sp, t + m * G);
        T K[6];
#pragma unroll
        for (int q = 0; q < 6; q++) K[q] = A0[q] + x3 * (A1[q] + x3 * A2[q]);
        const T k00 = K[0], k01 = K[1], k02 = K[2], k11 = K[3], k12 = K[4], k22 = K[5];
        V z0, z1, z2;
        if (sp.dim == 2) {
            const T id = s / (k00 * k11 - k01 * k01);
            z0 = cscale(csub(cscale(u[0][m], k11), cscale(u[1][m], k01)), id);
            z1 = cscale(csub(cscale(u[1][m], k00), cscale(u[0][m], k01)), id);
            z2 = V{0, 0};
        } else {
            // inverse of the symmetric 3x3 by cofactors
            const T c00 = k11 * k22 - k12 * k12;
            const T c01 = k02 * k12 - k01 * k22;
            const T c02 = k01 * k12 - k02 * k11;
            const T c11 = k00 * k22 - k02 * k02;
            const T c12 = k02 * k01 - k00 * k12;
            const T c22 = k00 * k11 - k01 * k01;
            const T id = s / (k00 * c00 + k01 * c01 + k02 * c02);
            const V r0 = u[0][m], r1 = u[1][m], r2 = u[2][m];
            z0 = cscale(cadd(cadd(cscale(r0, c00), cscale(r1, c01)), cscale(r2, c02)), id);
            z1 = cscale(cadd(cadd(cscale(r0, c01), cscale(r1, c11)), cscale(r2, c12)), id);
            z2 = cscale(cadd(cadd(cscale(r0, c02), cscale(r1, c12)), cscale(r2, c22)), id);
        }
        // r . z by Parseval on the half spectrum: bins 0 < kx < n1/2 stand for themselves
        // and their mirrors (weight 2); the packed slot kx = 0 holds the kx = 0 and
        // kx = n1/2 planes, whose cross terms are imaginary (weight 1, real part)
        part += u[0][m].x * z0.x + u[0][m].y * z0.y + u[1][m].x * z1.x + u[1][m].y * z1.y + u[2][m].x * z2.x +
                u[2][m].y * z2.y;
        u[0][m] = z0;
        u[1][m] = z1;
        u[2][m] = z2;
    }
#pragma unroll
    for (int j = 0; j < 3; j++) {
        group_fft<L, R, +1>(u[j], t, lds, addr, twL);
#pragma unroll
        for (int m = 0; m < R; m++) st_nt<NM_NT(ZPRE, T)>(&at(j, m), u[j][m]);
    }
    if (partials) {
        const double pd = (kx == 0 ? 1.0 : 2.0) * (double)part;
        double tot = 0.0;
        if (blockDim.x >= 64) {
            __shared__ double red[BLK / 64 > 0 ? BLK / 64 : 1];
            const double w = wave_sum(pd);
            if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = w;
            __syncthreads();
            if (threadIdx.x == 0)
                for (int i = 0; i < (int)(blockDim.x / 64); i++) tot += red[i];
        } else {
            // a block narrower than a wavefront (small 2D grids): no cross-lane shuffles
            __shared__ double red1[64];
            red1[threadIdx.x] = pd;
            __syncthreads();
            if (threadIdx.x == 0)
                for (int i = 0; i < (int)blockDim.x; i++) tot += red1[i];
        }
        if (threadIdx.x == 0)
            partials[((long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = tot;
    }
}

// ---------------------------------------------------------------------------
// Axis-wise derivative stages of the operator (see ColOp).  Data are x-spectral
// and real in y and z, so D_x is the multiplier i xi1 and D_y, D_z are round
// trips along one axis: forward FFT, i xi / n, inverse FFT.  Every element is
// read and written by the thread that owns its row in the FFT register layout.
// ---------------------------------------------------------------------------
template <typename T, int L, int R, int OP, int BLK, int TXC, bool PF>
__global__ __launch_bounds__(BLK) void k_colop(cx_t<T>* __restrict__ S, cx_t<T>* __restrict__ S2, long rowstride,
                                               long cs, int TXr, SpecParams sp, const cx_t<T>* __restrict__ tw)
{
    if (stopped(sp.stop)) return;
    using V = cx_t<T>;
    constexpr int G = L / R;
    constexpr bool YAX = (OP == YOP_DERIV || OP == YOP_DIV);
    const int TX = TXC > 0 ? TXC : TXr;
    __shared__ V lds[BLK * R];
    __shared__ V twsm[L > 1 ? L : 2];
    stage_twiddles<L>(twsm, tw);
    __syncthreads();
    const int tid = threadIdx.x, c = tid % TX, t = tid / TX;
    const int M = sp.n1 / 2;
    const int kx = blockIdx.x * TX + c;
    // y stages: block = (kx tile, z plane), rows along y at stride M;
    // z stages: block = (kx tile, y row), rows along z at the plane stride.
    // rowstride is the plane (kz) stride of the layout
    const long start = YAX ? (long)blockIdx.y * rowstride : (long)blockIdx.y * M;
    const long step = YAX ? (long)M : rowstride;
#if NM_COL_OFF32
    // uniform tile bases (scalar registers) plus 32-bit per-lane byte offsets
    // several fields at once: field blockIdx.z, spectra sp.bs elements apart
    V* const s1 = S + (long)blockIdx.z * sp.bs + start + (long)blockIdx.x * TX;
    V* const s2 = S2 + (long)blockIdx.z * sp.bs + start + (long)blockIdx.x * TX;
    const uint32_t lane = (uint32_t)(c * sizeof(V)) + (uint32_t)t * (uint32_t)(step * sizeof(V));
    const uint32_t mstep = (uint32_t)(G * step * sizeof(V));
#else
    V* s1 = S + (long)blockIdx.z * sp.bs + start + kx;
    V* s2 = S2 + (long)blockIdx.z * sp.bs + start + kx;
#endif
    ColAddrT<TXC> addr{c, TX};
    const V* twL = twsm;
    const T xi1 = (T)freq_x(sp, kx);
    const int n = YAX ? sp.n2 : sp.n3;
    const double kax = YAX ? sp.k2 * sp.inv_n2 : sp.k3 * sp.inv_n3;
    T mul[R];
    if (sp.mfreq) {
        const double* mf = sp.mfreq + sp.n1 + (YAX ? 0 : sp.n2);
        const double inv_n = YAX ? sp.inv_n2 : sp.inv_n3;
#pragma unroll
        for (int m = 0; m < R; m++) mul[m] = (T)(mf[t + m * G] * inv_n);
    } else {
#pragma unroll
        for (int m = 0; m < R; m++) mul[m] = (T)(kax * freq_index(t + m * G, n));
    }
#if NM_COL_OFF32
    auto ld = [&](const V* base, int comp, V (&v)[R]) {
        const char* p = (const char*)(base + comp * cs);
#pragma unroll
        for (int m = 0; m < R; m++) v[m] = ld_nt<NM_COLOP_OP_NT(OP, T)>((const V*)(p + (lane + (uint32_t)m * mstep)));
    };
    auto st = [&](V* base, int comp, const V (&v)[R]) {
        char* p = (char*)(base + comp * cs);
#pragma unroll
        for (int m = 0; m < R; m++) st_nt<NM_COLOP_OP_NT(OP, T)>((V*)(p + (lane + (uint32_t)m * mstep)), v[m]);
    };
#else
    auto ld = [&](const V* col, int comp, V (&v)[R]) {
#pragma unroll
        for (int m = 0; m < R; m++) v[m] = ld_nt<NM_COLOP_OP_NT(OP, T)>(col + comp * cs + (long)(t + m * G) * step);
    };
    auto st = [&](V* col, int comp, const V (&v)[R]) {
#pragma unroll
        for (int m = 0; m < R; m++) st_nt<NM_COLOP_OP_NT(OP, T)>(col + comp * cs + (long)(t + m * G) * step, v[m]);
    };
#endif
    // v <- D v along the column (forward FFT, i xi / n, inverse FFT)
    auto deriv = [&](V (&v)[R]) {
        group_fft<L, R, -1>(v, t, lds, addr, twL);
#pragma unroll
        for (int m = 0; m < R; m++) v[m] = ZOps<T>::iscale(v[m], mul[m]);
        group_fft<L, R, +1>(v, t, lds, addr, twL);
    };
    // Software-pipelined order (PF): the loads of the next operands are issued before a
    // transform so that they are in flight while it runs (the LDS barriers of the
    // transforms do not wait on global loads); it holds up to three operand tiles.
    if constexpr (PF && OP == YOP_DERIV) {
        V cur[R], nxt[R];
        ld(s1, 0, nxt);
#pragma unroll
        for (int j = 0; j < 3; j++) {
#pragma unroll
            for (int m = 0; m < R; m++) cur[m] = nxt[m];
            if (j < 2) ld(s1, j + 1, nxt);
            deriv(cur);
            st(s1, 3 + j, cur);
        }
    } else if constexpr (PF && OP == YOP_DIV) {
        // sigma Voigt 0..5 = s11 s22 s33 s23 s13 s12
        V a[R], b[R], c[R];
        ld(s2, 1, a); // s22
        ld(s2, 5, b); // s12
        ld(s2, 0, c); // s11
        deriv(a);
#pragma unroll
        for (int m = 0; m < R; m++) a[m] = cadd(a[m], ZOps<T>::iscale(b[m], xi1));
        st(s1, 1, a);
        ld(s2, 3, a); // s23
        deriv(b);
#pragma unroll
        for (int m = 0; m < R; m++) b[m] = cadd(b[m], ZOps<T>::iscale(c[m], xi1));
        st(s1, 0, b);
        ld(s2, 4, c); // s13
        deriv(a);
#pragma unroll
        for (int m = 0; m < R; m++) a[m] = cadd(a[m], ZOps<T>::iscale(c[m], xi1));
        st(s1, 2, a);
    } else if constexpr (PF && OP == ZOP_STRAIN) {
        const T sc = (T)sp.inv_n1;
        V a[R], b[R], c[R];
        ld(s1, 0, a); // U1
        ld(s1, 2, b); // U3
        ld(s1, 1, c); // U2
        {
            V d[R];
#pragma unroll
            for (int m = 0; m < R; m++) d[m] = cscale(ZOps<T>::iscale(a[m], xi1), sc);
            st(s2, 0, d); // eps11
        }
        deriv(a); // D_z U1
#pragma unroll
        for (int m = 0; m < R; m++) a[m] = cscale(cadd(a[m], ZOps<T>::iscale(b[m], xi1)), sc);
        st(s2, 4, a); // g13
        ld(s1, 3, a); // D_y U1
        deriv(b);     // D_z U3
#pragma unroll
        for (int m = 0; m < R; m++) b[m] = cscale(b[m], sc);
        st(s2, 2, b); // eps33
        ld(s1, 5, b); // D_y U3
#pragma unroll
        for (int m = 0; m < R; m++) a[m] = cscale(cadd(a[m], ZOps<T>::iscale(c[m], xi1)), sc);
        st(s2, 5, a); // g12
        ld(s1, 4, a); // D_y U2
        deriv(c);     // D_z U2
#pragma unroll
        for (int m = 0; m < R; m++) c[m] = cscale(cadd(c[m], b[m]), sc);
        st(s2, 3, c); // g23
#pragma unroll
        for (int m = 0; m < R; m++) a[m] = cscale(a[m], sc);
        st(s2, 1, a); // eps22
    } else if constexpr (PF && OP == ZOP_DIVZ) {
        const T cd = (T)(-sp.bdt2 * sp.inv_n1);
        constexpr int SRC[3] = {4, 3, 2};
        V v[R], w[R], vn[R];
        ld(s2, SRC[0], v);
        ld(s1, 0, w);
#pragma unroll
        for (int j = 0; j < 3; j++) {
            if (j < 2) ld(s2, SRC[j + 1], vn);
            deriv(v);
#pragma unroll
            for (int m = 0; m < R; m++) v[m] = cscale(cadd(v[m], w[m]), cd);
            st(s1, j, v);
            if (j < 2) {
                ld(s1, j + 1, w);
#pragma unroll
                for (int m = 0; m < R; m++) v[m] = vn[m];
            }
        }
    } else if constexpr (OP == YOP_DERIV) {
#pragma unroll 1
        for (int j = 0; j < 3; j++) {
            V v[R];
            ld(s1, j, v);
            deriv(v);
            st(s1, 3 + j, v);
        }
    } else if constexpr (OP == YOP_DIV) {
        // sigma Voigt 0..5 = s11 s22 s33 s23 s13 s12; five components are read once each
        // (s12 feeds both D_y s12 and i xi1 s12)
        V s12[R];
        {
            V v[R], w[R];
            ld(s2, 5, v);
#pragma unroll
            for (int m = 0; m < R; m++) s12[m] = v[m];
            deriv(v);
            ld(s2, 0, w);
#pragma unroll
            for (int m = 0; m < R; m++) v[m] = cadd(v[m], ZOps<T>::iscale(w[m], xi1));
            st(s1, 0, v);
        }
        {
            V v[R];
            ld(s2, 1, v);
            deriv(v);
#pragma unroll
            for (int m = 0; m < R; m++) v[m] = cadd(v[m], ZOps<T>::iscale(s12[m], xi1));
            st(s1, 1, v);
        }
        {
            V v[R], w[R];
            ld(s2, 3, v);
            deriv(v);
            ld(s2, 4, w);
#pragma unroll
            for (int m = 0; m < R; m++) v[m] = cadd(v[m], ZOps<T>::iscale(w[m], xi1));
            st(s1, 2, v);
        }
    } else if constexpr (OP == ZOP_STRAIN) {
        const T sc = (T)sp.inv_n1;
        V a[R], b[R];
        // eps11 = i xi1 U1 ; A = D_z U1
        ld(s1, 0, a);
#pragma unroll
        for (int m = 0; m < R; m++) b[m] = cscale(ZOps<T>::iscale(a[m], xi1), sc);
        st(s2, 0, b);
        deriv(a);
        // g13 = D_z U1 + i xi1 U3 ; eps33 = D_z U3
        ld(s1, 2, b);
#pragma unroll
        for (int m = 0; m < R; m++) a[m] = cscale(cadd(a[m], ZOps<T>::iscale(b[m], xi1)), sc);
        st(s2, 4, a);
        deriv(b);
#pragma unroll
        for (int m = 0; m < R; m++) b[m] = cscale(b[m], sc);
        st(s2, 2, b);
        // g23 = D_z U2 + D_y U3 ; g12 = D_y U1 + i xi1 U2 ; eps22 = D_y U2
        ld(s1, 1, a);
#pragma unroll
        for (int m = 0; m < R; m++) b[m] = a[m];
        deriv(b);
        {
            V d[R];
            ld(s1, 5, d);
#pragma unroll
            for (int m = 0; m < R; m++) d[m] = cscale(cadd(b[m], d[m]), sc);
            st(s2, 3, d);
            ld(s1, 3, d);
#pragma unroll
            for (int m = 0; m < R; m++) d[m] = cscale(cadd(d[m], ZOps<T>::iscale(a[m], xi1)), sc);
            st(s2, 5, d);
            ld(s1, 4, d);
#pragma unroll
            for (int m = 0; m < R; m++) d[m] = cscale(d[m], sc);
            st(s2, 1, d);
        }
    } else {
        // q_j = -beta dt^2 / n1 (Q_j + D_z sigma_j3): sigma_13 = S2[4], sigma_23 = S2[3], sigma_33 = S2[2]
        const T cd = (T)(-sp.bdt2 * sp.inv_n1);
        constexpr int SRC[3] = {4, 3, 2};
#pragma unroll
        for (int j = 0; j < 3; j++) {
            V v[R], w[R];
            ld(s2, SRC[j], v);
            deriv(v);
            ld(s1, j, w);
#pragma unroll
            for (int m = 0; m < R; m++) v[m] = cscale(cadd(v[m], w[m]), cd);
            st(s1, j, v);
        }
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static inline int radix_x(int M) { return M >= 8 ? 8 : M; }

// Radix of the x-direction stress pass in FP64 (it holds six components per thread).
#ifndef NM_STRESS_R64
#define NM_STRESS_R64 4
#endif
#ifndef NM_STRESS_R32
#define NM_STRESS_R32 4
#endif

int xfwd_blocks(int n1, long nlines)
{
    const int M = n1 / 2, G = M / radix_x(M), LPB = kBlock / G;
    return (int)((nlines + LPB - 1) / LPB);
}
int xinv_blocks(int n1, long nlines) { return xfwd_blocks(n1, nlines); }

#define NM_SIZE_SWITCH(n, ...)                                                                                         \
    switch (n) {                                                                                                       \
    case 8: { constexpr int NN = 8; __VA_ARGS__; } break;                                                              \
    case 16: { constexpr int NN = 16; __VA_ARGS__; } break;                                                            \
    case 32: { constexpr int NN = 32; __VA_ARGS__; } break;                                                            \
    case 64: { constexpr int NN = 64; __VA_ARGS__; } break;                                                            \
    case 128: { constexpr int NN = 128; __VA_ARGS__; } break;                                                          \
    case 256: { constexpr int NN = 256; __VA_ARGS__; } break;                                                          \
    case 512: { constexpr int NN = 512; __VA_ARGS__; } break;                                                          \
    default: return -1;                                                                                                \
    }

template <typename T> int launch_xfwd(int mode, int n1, const XFwdArgs& a, const void* tw, hipStream_t s)
{
    const int blocks = xfwd_blocks(n1, a.nlines);
    const cx_t<T>* t = (const cx_t<T>*)tw;
    NM_SIZE_SWITCH(n1, {
        constexpr int M = NN / 2, R = (M >= 8 ? 8 : M);
        if (mode == XF_PLAIN) hipLaunchKernelGGL((k_xfwd<T, NN, R, XF_PLAIN>), dim3(blocks), dim3(kBlock), 0, s, a, t);
        else if (mode == XF_EXPLICIT)
            hipLaunchKernelGGL((k_xfwd<T, NN, R, XF_EXPLICIT>), dim3(blocks), dim3(kBlock), 0, s, a, t);
        else hipLaunchKernelGGL((k_xfwd<T, NN, R, XF_UPDATE>), dim3(blocks), dim3(kBlock), 0, s, a, t);
    })
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <typename T> int launch_xinv(int mode, int n1, const XInvArgs& a, const void* tw, hipStream_t s)
{
    const int blocks = xinv_blocks(n1, a.nlines);
    const cx_t<T>* t = (const cx_t<T>*)tw;
    NM_SIZE_SWITCH(n1, {
        constexpr int M = NN / 2, R = (M >= 8 ? 8 : M);
        if (mode == XI_PLAIN) hipLaunchKernelGGL((k_xinv<T, NN, R, XI_PLAIN>), dim3(blocks), dim3(kBlock), 0, s, a, t);
        else if (mode == XI_OPERATOR)
            hipLaunchKernelGGL((k_xinv<T, NN, R, XI_OPERATOR>), dim3(blocks), dim3(kBlock), 0, s, a, t);
        else if (mode == XI_EXPLICIT)
            hipLaunchKernelGGL((k_xinv<T, NN, R, XI_EXPLICIT>), dim3(blocks), dim3(kBlock), 0, s, a, t);
        else hipLaunchKernelGGL((k_xinv<T, NN, R, XI_PRECOND>), dim3(blocks), dim3(kBlock), 0, s, a, t);
    })
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <typename T> int launch_xpupdate(int n1, const XInvArgs& a, const void* tw, hipStream_t s)
{
    const int blocks = xinv_blocks(n1, a.nlines);
    const cx_t<T>* t = (const cx_t<T>*)tw;
    NM_SIZE_SWITCH(n1, {
        constexpr int M = NN / 2, R = (M >= 8 ? 8 : M);
        hipLaunchKernelGGL((k_xpupdate<T, NN, R>), dim3(blocks), dim3(kBlock), 0, s, a, t);
    })
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <typename T>
int launch_xstress(int n1, void* spec, const SpecLayout& lay, const uint16_t* phase, const void* C21, const void* tw,
                   hipStream_t s)
{
    const long lpc = (long)lay.n2 * lay.n3 * lay.nb;
    const cx_t<T>* t = (const cx_t<T>*)tw;
    NM_SIZE_SWITCH(n1, {
        constexpr int M = NN / 2;
        constexpr int RQ = sizeof(T) == 8 ? (NN == 512 ? NM_STRESS512_R64 : NM_STRESS_R64) : NM_STRESS_R32;
        constexpr int R0 = M >= RQ ? RQ : M;
        constexpr int R = R0 * 64 >= M ? R0 : M / 64; // a line stays inside one wavefront
        constexpr int G = M / R, LPB = kBlock / G;
        const int blocks = (int)((lpc + LPB - 1) / LPB);
        hipLaunchKernelGGL((k_xstress<T, NN, R>), dim3(blocks), dim3(kBlock), 0, s, (cx_t<T>*)spec, lay, phase,
                           (const T*)C21, t);
    })
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

// Radix and block size of the column passes.  The y pass holds one component
// per thread (radix 16: one LDS exchange for L = 256); the fused z kernels hold
// three components, so FP64 uses a smaller radix to bound register pressure.
#ifndef NM_ZSPEC_R64
#define NM_ZSPEC_R64 8
#endif
#ifndef NM_ZSPEC_R32
#define NM_ZSPEC_R32 8
#endif
#ifndef NM_ZSPEC_BLK64
#define NM_ZSPEC_BLK64 256
#endif
#ifndef NM_ZSPEC_BLK32
#define NM_ZSPEC_BLK32 256
#endif

// Block sizes of the column passes on 512-long columns: a block holds BLK / G columns of G
// threads each, so a larger block keeps the rows of a tile wide (coalesced) when G is large.
// Measured at 512^3 (pass times in us, 256-thread blocks -> these): FP32 z strain 1885 -> 1410,
// z divergence 1352 -> 1098, y divergence 1050 -> 906, preconditioner y passes 759/765 ->
// 606/607 and z pass 1544 -> 1086 (radix 16); FP64 z strain 3220 -> 2810, z divergence
// 2569 -> 2127, preconditioner z pass 2994 -> 2518.  The FP64 y passes stay at 256 (512 was
// 2-5% slower).  LDS per block: up to 64 KB of exchange buffer plus the twiddle table.
#ifndef NM_COL512_BLK32
#define NM_COL512_BLK32 512
#endif
#ifndef NM_YPASS512_BLK32
#define NM_YPASS512_BLK32 512
#endif
#ifndef NM_ZSPEC512_BLK32
#define NM_ZSPEC512_BLK32 512
#endif
#ifndef NM_ZSPEC512_BLK64
#define NM_ZSPEC512_BLK64 512
#endif
#ifndef NM_COL512_ZBLK64
#define NM_COL512_ZBLK64 512
#endif
#ifndef NM_YPASS512_BLK64
#define NM_YPASS512_BLK64 256
#endif
#ifndef NM_ZSPEC512_R32
#define NM_ZSPEC512_R32 16
#endif

template <int L> constexpr int ypass_radix() { return L >= 16 ? 16 : L; }
template <typename T, int L> constexpr int ypass_block()
{
    return L == 512 ? (sizeof(T) == 4 ? NM_YPASS512_BLK32 : NM_YPASS512_BLK64) : 256;
}
template <typename T, int L> constexpr int zspec_radix()
{
    return L < 8 ? L
                 : (sizeof(T) == 8 ? (NM_ZSPEC_R64 < L ? NM_ZSPEC_R64 : L)
                                   : (L == 512 ? NM_ZSPEC512_R32 : (NM_ZSPEC_R32 < L ? NM_ZSPEC_R32 : L)));
}
template <typename T, int L> constexpr int zspec_block()
{
    return L == 512 ? (sizeof(T) == 8 ? NM_ZSPEC512_BLK64 : NM_ZSPEC512_BLK32)
                    : (sizeof(T) == 8 ? NM_ZSPEC_BLK64 : NM_ZSPEC_BLK32);
}


template <typename T>
int launch_ypass(int dir, int ncomp, const SpecLayout& lay, void* spec, const void* tw, hipStream_t s)
{
    const int M = lay.M, n3 = lay.n3;
    const cx_t<T>* t = (const cx_t<T>*)tw;
    NM_SIZE_SWITCH(lay.n2, {
        constexpr int R = ypass_radix<NN>();
        constexpr int G = NN / R;
        constexpr int BLK = ypass_block<T, NN>();
        constexpr int TXP = BLK / G;
        const int TX = M >= TXP ? TXP : M;
        dim3 grid(M / TX, n3, ncomp), block(TX * G);
        cx_t<T>* d = (cx_t<T>*)spec;
        if (M >= TXP) {
            if (dir < 0)
                hipLaunchKernelGGL((k_ypass<T, NN, R, -1, BLK, TXP>), grid, block, 0, s, d, (long)M, lay.ps, lay.cs, TX, t, lay.stop, lay.bs);
            else
                hipLaunchKernelGGL((k_ypass<T, NN, R, +1, BLK, TXP>), grid, block, 0, s, d, (long)M, lay.ps, lay.cs, TX, t, lay.stop, lay.bs);
        } else {
            if (dir < 0)
                hipLaunchKernelGGL((k_ypass<T, NN, R, -1, BLK, 0>), grid, block, 0, s, d, (long)M, lay.ps, lay.cs, TX, t, lay.stop, lay.bs);
            else
                hipLaunchKernelGGL((k_ypass<T, NN, R, +1, BLK, 0>), grid, block, 0, s, d, (long)M, lay.ps, lay.cs, TX, t, lay.stop, lay.bs);
        }
    })
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <typename T, int L, int BLK, int TXC>
static void zprecond_dispatch(dim3 grid, dim3 block, hipStream_t s, cx_t<T>* spec, const SpecLayout& lay, int TX,
                              const SpecParams& sp, const cx_t<T>* t, double* partials)
{
    constexpr int R = zspec_radix<T, L>();
    hipLaunchKernelGGL((k_zprecond<T, L, R, BLK, TXC>), grid, block, 0, s, spec, lay.cs, lay.ps, TX, sp, t,
                       partials);
}

template <typename T> int zprecond_blocks(const SpecParams& sp)
{
    const int M = sp.n1 / 2;
    if (sp.n3 == 1) {
        constexpr int BLK = zspec_block<T, 1>();
        const int TX = M < BLK ? M : BLK;
        return (M / TX) * sp.n2;
    }
    int nb = 0;
    [&]() -> int {
        NM_SIZE_SWITCH(sp.n3, {
            constexpr int BLK = zspec_block<T, NN>();
            constexpr int G = NN / zspec_radix<T, NN>();
            constexpr int TXP = BLK / G;
            nb = (M >= TXP ? M / TXP : 1) * sp.n2;
        })
        return 0;
    }();
    return nb;
}

template <typename T>
int launch_zprecond(const SpecParams& sp, const SpecLayout& lay, void* spec, const void* tw, hipStream_t s,
                    double* partials)
{
    const int M = sp.n1 / 2;
    const cx_t<T>* t = (const cx_t<T>*)tw;
    cx_t<T>* d = (cx_t<T>*)spec;
    if (sp.n3 == 1) {
        constexpr int BLK = zspec_block<T, 1>();
        const int TX = M < BLK ? M : BLK;
        zprecond_dispatch<T, 1, BLK, 0>(dim3(M / TX, sp.n2, sp.bk), dim3(TX), s, d, lay, TX, sp, t, partials);
    } else {
        NM_SIZE_SWITCH(sp.n3, {
            constexpr int BLK = zspec_block<T, NN>();
            constexpr int G = NN / zspec_radix<T, NN>();
            constexpr int TXP = BLK / G;
            if (M >= TXP)
                zprecond_dispatch<T, NN, BLK, TXP>(dim3(M / TXP, sp.n2, sp.bk), dim3(TXP * G), s, d, lay, TXP, sp, t,
                                                    partials);
            else
                zprecond_dispatch<T, NN, BLK, 0>(dim3(1, sp.n2, sp.bk), dim3(M * G), s, d, lay, M, sp, t, partials);
        })
    }
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

#ifndef NM_COLOP_R64
#define NM_COLOP_R64 16
#endif
// Software-pipelined column operators (three operand tiles per thread).
#ifndef NM_COLOP_PF32
#define NM_COLOP_PF32 1
#endif
#ifndef NM_COLOP_PF64
#define NM_COLOP_PF64 0
#endif
template <typename T, int L> constexpr int colop_radix()
{
    return L < 16 ? L : (sizeof(T) == 8 ? (NM_COLOP_R64 < L ? NM_COLOP_R64 : L) : 16);
}

#ifndef NM_COL256_YBLK32
#define NM_COL256_YBLK32 256
#endif
#ifndef NM_COL256_ZBLK32
#define NM_COL256_ZBLK32 256
#endif
template <typename T, int L, int OP> constexpr int colop_block()
{
    return L == 512 ? (sizeof(T) == 4 ? NM_COL512_BLK32
                                      : ((OP == ZOP_STRAIN || OP == ZOP_DIVZ) ? NM_COL512_ZBLK64 : 256))
                    : ((L == 256 && sizeof(T) == 4) ? ((OP == ZOP_STRAIN || OP == ZOP_DIVZ) ? NM_COL256_ZBLK32
                                                                                            : NM_COL256_YBLK32)
                                                    : 256);
}

template <typename T, int L, int TXC>
static void colop_dispatch(int op, dim3 grid, dim3 block, hipStream_t s, cx_t<T>* S, cx_t<T>* S2, long rowstride,
                           long cs, int TX, const SpecParams& sp, const cx_t<T>* t)
{
    constexpr int R = colop_radix<T, L>();
    constexpr bool PF = sizeof(T) == 8 ? NM_COLOP_PF64 : NM_COLOP_PF32;
    switch (op) {
    case YOP_DERIV:
        hipLaunchKernelGGL((k_colop<T, L, R, YOP_DERIV, colop_block<T, L, YOP_DERIV>(), TXC, PF>), grid, block, 0, s, S,
                           S2, rowstride, cs, TX, sp, t);
        break;
    case YOP_DIV:
        hipLaunchKernelGGL((k_colop<T, L, R, YOP_DIV, colop_block<T, L, YOP_DIV>(), TXC, PF>), grid, block, 0, s, S, S2,
                           rowstride, cs, TX, sp, t);
        break;
    case ZOP_STRAIN:
        hipLaunchKernelGGL((k_colop<T, L, R, ZOP_STRAIN, colop_block<T, L, ZOP_STRAIN>(), TXC, PF>), grid, block, 0, s,
                           S, S2, rowstride, cs, TX, sp, t);
        break;
    default:
        hipLaunchKernelGGL((k_colop<T, L, R, ZOP_DIVZ, colop_block<T, L, ZOP_DIVZ>(), TXC, PF>), grid, block, 0, s, S,
                           S2, rowstride, cs, TX, sp, t);
        break;
    }
}

template <typename T>
int launch_colop(int op, const SpecParams& sp, const SpecLayout& lay, void* S, void* S2, const void* tw,
                 hipStream_t s)
{
    const int M = lay.M;
    const cx_t<T>* t = (const cx_t<T>*)tw;
    cx_t<T>* a = (cx_t<T>*)S;
    cx_t<T>* b = (cx_t<T>*)S2;
    const bool yax = (op == YOP_DERIV || op == YOP_DIV);
    const int L = yax ? lay.n2 : lay.n3;
    const int planes = yax ? lay.n3 : lay.n2;
    if (L == 1) {
        const int TX = M < 256 ? M : 256;
        colop_dispatch<T, 1, 0>(op, dim3(M / TX, planes, sp.bk), dim3(TX), s, a, b, lay.ps, lay.cs, TX, sp, t);
    } else {
        NM_SIZE_SWITCH(L, {
            constexpr int G = NN / colop_radix<T, NN>();
            // y and z operators may take different block sizes (and so tile widths)
            constexpr int TXY = colop_block<T, NN, YOP_DERIV>() / G;
            constexpr int TXZ = colop_block<T, NN, ZOP_STRAIN>() / G;
            if (yax ? M >= TXY : M >= TXZ) {
                if (yax)
                    colop_dispatch<T, NN, TXY>(op, dim3(M / TXY, planes, sp.bk), dim3(TXY * G), s, a, b, lay.ps, lay.cs,
                                               TXY, sp, t);
                else
                    colop_dispatch<T, NN, TXZ>(op, dim3(M / TXZ, planes, sp.bk), dim3(TXZ * G), s, a, b, lay.ps, lay.cs,
                                               TXZ, sp, t);
            } else {
                colop_dispatch<T, NN, 0>(op, dim3(1, planes, sp.bk), dim3(M * G), s, a, b, lay.ps, lay.cs, M, sp, t);
            }
        })
    }
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

#define NM_INST(T)                                                                                                     \
    template int launch_xfwd<T>(int, int, const XFwdArgs&, const void*, hipStream_t);                                  \
    template int launch_xinv<T>(int, int, const XInvArgs&, const void*, hipStream_t);                                  \
    template int launch_xpupdate<T>(int, const XInvArgs&, const void*, hipStream_t);                                   \
    template int launch_xstress<T>(int, void*, const SpecLayout&, const uint16_t*, const void*, const void*,          \
                                   hipStream_t);                                                                       \
    template int launch_ypass<T>(int, int, const SpecLayout&, void*, const void*, hipStream_t);                        \
    template int launch_zprecond<T>(const SpecParams&, const SpecLayout&, void*, const void*, hipStream_t, double*); \
    template int zprecond_blocks<T>(const SpecParams&);                                                             \
    template int launch_colop<T>(int, const SpecParams&, const SpecLayout&, void*, void*, const void*, hipStream_t);
NM_INST(double)
NM_INST(float)

} // namespace nm
