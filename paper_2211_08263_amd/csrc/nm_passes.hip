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
// Passes of one operator apply q = A p (9 kernels, every pointwise stage
// fused into a transform pass):
//   x-fwd(3) | y-fwd(3) | z-fwd, grad, z-inv (3->6) | y-inv(6) |
//   x-inv, sigma = C:eps, x-fwd (6) | y-fwd(6) | z-fwd, div, z-inv (6->3) |
//   y-inv(3) | x-inv + rho p (3).
#include "nm_common.h"
#include "nm_fft.h"
#include "nm_passes.h"

namespace nm {

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

// ---------------------------------------------------------------------------
// x direction: real lines of N1 points, M = N1/2 complex points per line
// ---------------------------------------------------------------------------
template <typename T, int N1, int R, int MODE>
__global__ __launch_bounds__(kBlock) void k_xfwd(XFwdArgs a, const cx_t<T>* __restrict__ tw)
{
    using V = cx_t<T>;
    constexpr int M = N1 / 2, G = M / R, LPB = kBlock / G, LP = M + M / R;
    __shared__ V lds[LPB * LP];
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
            for (int m = 0; m < R; m++) v[m] = src[t + m * G];
        } else if constexpr (MODE == XF_PUPDATE) {
            const V* z = (const V*)a.src + off;
            V* p = (V*)a.p + off;
            const T beta = (T)a.scal[S_BETA];
            const bool first = a.scal[S_FIRST] != 0.0;
#pragma unroll
            for (int m = 0; m < R; m++) {
                const int i = t + m * G;
                V zz = z[i];
                V pp = zz;
                if (!first) {
                    V po = p[i];
                    pp = V{zz.x + beta * po.x, zz.y + beta * po.y};
                }
                p[i] = pp;
                v[m] = pp;
            }
        } else {
            const T alpha = (T)a.scal[S_ALPHA];
            V* x = (V*)a.x + off;
            V* r = (V*)a.r + off;
            const V* p = (const V*)a.p + off;
            const V* q = (const V*)a.q + off;
#pragma unroll
            for (int m = 0; m < R; m++) {
                const int i = t + m * G;
                V pp = p[i], qq = q[i], xx = x[i], rr = r[i];
                xx = V{xx.x + alpha * pp.x, xx.y + alpha * pp.y};
                rr = V{rr.x - alpha * qq.x, rr.y - alpha * qq.y};
                x[i] = xx;
                r[i] = rr;
                part += (double)rr.x * (double)rr.x + (double)rr.y * (double)rr.y;
                v[m] = rr;
            }
        }
    }
    LineAddr<R> addr{ll * LP};
    group_fft<M, R, -1>(v, t, lds, addr, tw + tw_offset(M));
#pragma unroll
    for (int m = 0; m < R; m++) lds[addr(t + m * G)] = v[m];
    __syncthreads();
    V mir[R];
#pragma unroll
    for (int m = 0; m < R; m++) mir[m] = lds[addr((M - (t + m * G)) & (M - 1))];
    const V* twN = tw + tw_offset(N1);
    if (valid) {
        V* out = (V*)a.spec + off;
#pragma unroll
        for (int m = 0; m < R; m++) {
            const int k = t + m * G;
            out[k] = r2c_post(k, v[m], mir[m], twN[k]);
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
    using V = cx_t<T>;
    constexpr int M = N1 / 2, G = M / R, LPB = kBlock / G, LP = M + M / R;
    __shared__ V lds[LPB * LP];
    const int tid = threadIdx.x, ll = tid / G, t = tid % G;
    const long line = (long)blockIdx.x * LPB + ll;
    const bool valid = line < a.nlines;
    const long off = line * M;
    V v[R];
#pragma unroll
    for (int m = 0; m < R; m++) v[m] = valid ? ((const V*)a.spec)[off + t + m * G] : V{0, 0};
    LineAddr<R> addr{ll * LP};
#pragma unroll
    for (int m = 0; m < R; m++) lds[addr(t + m * G)] = v[m];
    __syncthreads();
    const V* twN = tw + tw_offset(N1);
#pragma unroll
    for (int m = 0; m < R; m++) {
        const int k = t + m * G;
        V xm = lds[addr((M - k) & (M - 1))];
        v[m] = c2r_pre(k, v[m], xm, twN[k]);
    }
    __syncthreads();
    group_fft<M, R, +1>(v, t, lds, addr, tw + tw_offset(M));
    double part = 0.0;
    if (valid) {
        V* out = (V*)a.out + off;
        if constexpr (MODE == XI_PLAIN) {
#pragma unroll
            for (int m = 0; m < R; m++) out[t + m * G] = v[m];
        } else {
            const V* aux = (const V*)a.aux + off;
            const long vline = line % a.lines_per_comp;
            const bool zero_comp = (a.dim == 2) && (line / a.lines_per_comp == 2);
            const uint32_t* ph2 = (const uint32_t*)a.phase + vline * M;
            const uint16_t* mk2 = a.mask ? (const uint16_t*)a.mask + vline * M : nullptr;
            const T* rho = (const T*)a.rho;
#pragma unroll
            for (int m = 0; m < R; m++) {
                const int n = t + m * G;
                V au = aux[n];
                V o = v[m];
                if constexpr (MODE == XI_OPERATOR) {
                    const uint32_t ph = ph2[n];
                    o.x += rho[ph & 0xffffu] * au.x;
                    o.y += rho[ph >> 16] * au.y;
                }
                if (mk2) {
                    const uint16_t mm = mk2[n];
                    if (mm & 0x00ffu) o.x = 0;
                    if (mm & 0xff00u) o.y = 0;
                }
                if (zero_comp) o = V{0, 0};
                part += (double)au.x * (double)o.x + (double)au.y * (double)o.y;
                out[n] = o;
            }
        }
    }
    if constexpr (MODE != XI_PLAIN) {
        double s = block_sum256(part);
        if (threadIdx.x == 0 && a.partials) a.partials[blockIdx.x] = s;
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
__global__ __launch_bounds__(kBlock) void k_xstress(cx_t<T>* spec, long lpc, long NS, const uint16_t* __restrict__ phase,
                                                    const T* __restrict__ C21, const cx_t<T>* __restrict__ tw)
{
    using V = cx_t<T>;
    constexpr int M = N1 / 2, G = M / R, LPB = kBlock / G, LP = M + M / R;
    __shared__ V lds[LPB * LP];
    const int tid = threadIdx.x, ll = tid / G, t = tid % G;
    const long line = (long)blockIdx.x * LPB + ll;
    const bool valid = line < lpc;
    const long off = line * M;
    LineAddr<R> addr{ll * LP};
    const V* twN = tw + tw_offset(N1);
    const V* twM = tw + tw_offset(M);
    T e[6][2 * R];
#pragma unroll
    for (int c = 0; c < 6; c++) {
        V v[R];
#pragma unroll
        for (int m = 0; m < R; m++) v[m] = valid ? spec[c * NS + off + t + m * G] : V{0, 0};
#pragma unroll
        for (int m = 0; m < R; m++) lds[addr(t + m * G)] = v[m];
        __syncthreads();
#pragma unroll
        for (int m = 0; m < R; m++) {
            const int k = t + m * G;
            v[m] = c2r_pre(k, v[m], lds[addr((M - k) & (M - 1))], twN[k]);
        }
        __syncthreads();
        group_fft<M, R, +1>(v, t, lds, addr, twM);
#pragma unroll
        for (int m = 0; m < R; m++) {
            e[c][2 * m] = v[m].x;
            e[c][2 * m + 1] = v[m].y;
        }
    }
    if (valid) {
        const uint32_t* ph2 = (const uint32_t*)phase + line * M;
#pragma unroll
        for (int m = 0; m < R; m++) {
            const uint32_t ph = ph2[t + m * G];
#pragma unroll
            for (int h = 0; h < 2; h++) {
                const T* c = C21 + 21 * (h ? (ph >> 16) : (ph & 0xffffu));
                T ee[6], ss[6];
#pragma unroll
                for (int q = 0; q < 6; q++) ee[q] = e[q][2 * m + h];
                voigt_stress(c, ee, ss);
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
        group_fft<M, R, -1>(v, t, lds, addr, twM);
#pragma unroll
        for (int m = 0; m < R; m++) lds[addr(t + m * G)] = v[m];
        __syncthreads();
        V mir[R];
#pragma unroll
        for (int m = 0; m < R; m++) mir[m] = lds[addr((M - (t + m * G)) & (M - 1))];
        __syncthreads();
        if (valid) {
#pragma unroll
            for (int m = 0; m < R; m++) {
                const int k = t + m * G;
                spec[c * NS + off + k] = r2c_post(k, v[m], mir[m], twN[k]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// y and z directions: tiles of TX consecutive kx columns, L points each.
// ---------------------------------------------------------------------------
template <int R> struct ColAddrRT {
    int c, tx;
    __device__ __forceinline__ int operator()(int p) const { return p * tx + c + p / R; }
};

template <typename T, int L, int R, int DIR>
__global__ __launch_bounds__(kBlock) void k_ypass(cx_t<T>* data, long colstride, long planestride, long NS, int TX,
                                                  const cx_t<T>* __restrict__ tw)
{
    using V = cx_t<T>;
    constexpr int G = L / R;
    __shared__ V lds[kBlock * R + L / R + 1]; // TX * L <= 256 R, plus one pad per R rows
    const int tid = threadIdx.x, c = tid % TX, t = tid / TX;
    V* col = data + blockIdx.z * NS + blockIdx.y * planestride + (long)blockIdx.x * TX + c;
    V v[R];
#pragma unroll
    for (int m = 0; m < R; m++) v[m] = col[(long)(t + m * G) * colstride];
    ColAddrRT<R> addr{c, TX};
    group_fft<L, R, DIR>(v, t, lds, addr, tw + tw_offset(L));
#pragma unroll
    for (int m = 0; m < R; m++) col[(long)(t + m * G) * colstride] = v[m];
}

// Pointwise operators at frequency (xi1, xi2, xi3).
template <typename T> struct ZOps {
    using V = cx_t<T>;
    // i s (a): multiply by i and a real scale
    static __device__ __forceinline__ V iscale(V a, T s) { return V{-a.y * s, a.x * s}; }
};

template <typename T, int L, int R, int OP>
__global__ __launch_bounds__(kBlock) void k_zspec(cx_t<T>* data, long NS, int TX, SpecParams sp,
                                                  const cx_t<T>* __restrict__ tw)
{
    using V = cx_t<T>;
    constexpr int G = L / R;
    __shared__ V lds[kBlock * R + L / R + 1]; // TX * L <= 256 R, plus one pad per R rows
    const int tid = threadIdx.x, c = tid % TX, t = tid / TX;
    const int M = sp.n1 / 2;
    const int kx = blockIdx.x * TX + c, ky = blockIdx.y;
    const long colstride = (long)sp.n2 * M;
    V* col = data + (long)ky * M + kx;
    ColAddrRT<R> addr{c, TX};
    const V* twL = tw + tw_offset(L > 1 ? L : 2);
    const T xi1 = (T)(6.283185307179586476925286766559 * kx / sp.L1);
    const T xi2 = (T)freq_of(ky, sp.n2, sp.L2);
    T xi3[R];
#pragma unroll
    for (int m = 0; m < R; m++) xi3[m] = (T)freq_of(t + m * G, sp.n3, sp.L3);

    if constexpr (OP == ZOP_GRAD || OP == ZOP_PRECOND) {
        V u[3][R];
#pragma unroll
        for (int j = 0; j < 3; j++) {
#pragma unroll
            for (int m = 0; m < R; m++) u[j][m] = col[j * NS + (long)(t + m * G) * colstride];
            group_fft<L, R, -1>(u[j], t, lds, addr, twL);
        }
        if constexpr (OP == ZOP_GRAD) {
            const T s = (T)sp.inv_ntot;
#pragma unroll
            for (int e = 0; e < 6; e++) {
                V w[R];
#pragma unroll
                for (int m = 0; m < R; m++) {
                    const T x3 = xi3[m];
                    V a;
                    switch (e) {
                    case 0: a = cscale(u[0][m], xi1); break;
                    case 1: a = cscale(u[1][m], xi2); break;
                    case 2: a = cscale(u[2][m], x3); break;
                    case 3: a = cadd(cscale(u[1][m], x3), cscale(u[2][m], xi2)); break;
                    case 4: a = cadd(cscale(u[0][m], x3), cscale(u[2][m], xi1)); break;
                    default: a = cadd(cscale(u[0][m], xi2), cscale(u[1][m], xi1)); break;
                    }
                    w[m] = ZOps<T>::iscale(a, s);
                }
                group_fft<L, R, +1>(w, t, lds, addr, twL);
#pragma unroll
                for (int m = 0; m < R; m++) col[e * NS + (long)(t + m * G) * colstride] = w[m];
            }
        } else {
            // (beta dt^2 K(xi) + rhobar I)^-1, K = N(xi)^T Cbar N(xi)
            T C[6][6];
            {
                int o = 0;
#pragma unroll
                for (int a = 0; a < 6; a++)
#pragma unroll
                    for (int b = a; b < 6; b++) {
                        C[a][b] = (T)sp.Cbar[o];
                        C[b][a] = (T)sp.Cbar[o];
                        o++;
                    }
            }
            const T bdt2 = (T)sp.bdt2, rb = (T)sp.rhobar, s = (T)sp.inv_ntot;
#pragma unroll
            for (int m = 0; m < R; m++) {
                const T x1 = xi1, x2 = xi2, x3 = xi3[m];
                T CN[6][3];
#pragma unroll
                for (int a = 0; a < 6; a++) {
                    CN[a][0] = C[a][0] * x1 + C[a][4] * x3 + C[a][5] * x2;
                    CN[a][1] = C[a][1] * x2 + C[a][3] * x3 + C[a][5] * x1;
                    CN[a][2] = C[a][2] * x3 + C[a][3] * x2 + C[a][4] * x1;
                }
                T K[3][3];
#pragma unroll
                for (int j = 0; j < 3; j++) {
                    K[0][j] = bdt2 * (x1 * CN[0][j] + x3 * CN[4][j] + x2 * CN[5][j]);
                    K[1][j] = bdt2 * (x2 * CN[1][j] + x3 * CN[3][j] + x1 * CN[5][j]);
                    K[2][j] = bdt2 * (x3 * CN[2][j] + x2 * CN[3][j] + x1 * CN[4][j]);
                }
                K[0][0] += rb;
                K[1][1] += rb;
                K[2][2] += rb;
                V z0, z1, z2;
                if (sp.dim == 2) {
                    const T det = K[0][0] * K[1][1] - K[0][1] * K[1][0];
                    const T id = s / det;
                    z0 = cscale(csub(cscale(u[0][m], K[1][1]), cscale(u[1][m], K[0][1])), id);
                    z1 = cscale(csub(cscale(u[1][m], K[0][0]), cscale(u[0][m], K[1][0])), id);
                    z2 = V{0, 0};
                } else {
                    // inverse of the symmetric 3x3 by cofactors
                    const T c00 = K[1][1] * K[2][2] - K[1][2] * K[2][1];
                    const T c01 = K[0][2] * K[2][1] - K[0][1] * K[2][2];
                    const T c02 = K[0][1] * K[1][2] - K[0][2] * K[1][1];
                    const T c11 = K[0][0] * K[2][2] - K[0][2] * K[2][0];
                    const T c12 = K[0][2] * K[1][0] - K[0][0] * K[1][2];
                    const T c22 = K[0][0] * K[1][1] - K[0][1] * K[1][0];
                    const T det = K[0][0] * c00 + K[0][1] * (K[1][2] * K[2][0] - K[1][0] * K[2][2]) +
                                  K[0][2] * (K[1][0] * K[2][1] - K[1][1] * K[2][0]);
                    const T id = s / det;
                    const V r0 = u[0][m], r1 = u[1][m], r2 = u[2][m];
                    z0 = cscale(cadd(cadd(cscale(r0, c00), cscale(r1, c01)), cscale(r2, c02)), id);
                    z1 = cscale(cadd(cadd(cscale(r0, c01), cscale(r1, c11)), cscale(r2, c12)), id);
                    z2 = cscale(cadd(cadd(cscale(r0, c02), cscale(r1, c12)), cscale(r2, c22)), id);
                }
                u[0][m] = z0;
                u[1][m] = z1;
                u[2][m] = z2;
            }
#pragma unroll
            for (int j = 0; j < 3; j++) {
                group_fft<L, R, +1>(u[j], t, lds, addr, twL);
#pragma unroll
                for (int m = 0; m < R; m++) col[j * NS + (long)(t + m * G) * colstride] = u[j][m];
            }
        }
    } else {
        // divergence: q_j = -beta dt^2 i xi_k sigma_jk, accumulated over the 6 Voigt components
        V q[3][R];
#pragma unroll
        for (int j = 0; j < 3; j++)
#pragma unroll
            for (int m = 0; m < R; m++) q[j][m] = V{0, 0};
        const T s = (T)(-sp.bdt2 * sp.inv_ntot);
#pragma unroll
        for (int e = 0; e < 6; e++) {
            V w[R];
#pragma unroll
            for (int m = 0; m < R; m++) w[m] = col[e * NS + (long)(t + m * G) * colstride];
            group_fft<L, R, -1>(w, t, lds, addr, twL);
#pragma unroll
            for (int m = 0; m < R; m++) {
                const V is = ZOps<T>::iscale(w[m], s);
                const T x3 = xi3[m];
                switch (e) {
                case 0: q[0][m] = cadd(q[0][m], cscale(is, xi1)); break;
                case 1: q[1][m] = cadd(q[1][m], cscale(is, xi2)); break;
                case 2: q[2][m] = cadd(q[2][m], cscale(is, x3)); break;
                case 3:
                    q[1][m] = cadd(q[1][m], cscale(is, x3));
                    q[2][m] = cadd(q[2][m], cscale(is, xi2));
                    break;
                case 4:
                    q[0][m] = cadd(q[0][m], cscale(is, x3));
                    q[2][m] = cadd(q[2][m], cscale(is, xi1));
                    break;
                default:
                    q[0][m] = cadd(q[0][m], cscale(is, xi2));
                    q[1][m] = cadd(q[1][m], cscale(is, xi1));
                    break;
                }
            }
        }
#pragma unroll
        for (int j = 0; j < 3; j++) {
            group_fft<L, R, +1>(q[j], t, lds, addr, twL);
#pragma unroll
            for (int m = 0; m < R; m++) col[j * NS + (long)(t + m * G) * colstride] = q[j][m];
        }
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static inline int radix_x(int M) { return M >= 8 ? 8 : M; }
static inline int radix_stress(int M, bool dbl) { return dbl ? (M >= 4 ? 4 : M) : (M >= 8 ? 8 : M); }
static inline int radix_col(int L) { return L >= 8 ? 8 : L; }

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
        else if (mode == XF_PUPDATE)
            hipLaunchKernelGGL((k_xfwd<T, NN, R, XF_PUPDATE>), dim3(blocks), dim3(kBlock), 0, s, a, t);
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
        else hipLaunchKernelGGL((k_xinv<T, NN, R, XI_PRECOND>), dim3(blocks), dim3(kBlock), 0, s, a, t);
    })
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <typename T>
int launch_xstress(int n1, void* spec, long lpc, long NS, const uint16_t* phase, const void* C21, const void* tw,
                   hipStream_t s)
{
    const cx_t<T>* t = (const cx_t<T>*)tw;
    NM_SIZE_SWITCH(n1, {
        constexpr int M = NN / 2;
        constexpr int R = sizeof(T) == 8 ? (M >= 4 ? 4 : M) : (M >= 8 ? 8 : M);
        constexpr int G = M / R, LPB = kBlock / G;
        const int blocks = (int)((lpc + LPB - 1) / LPB);
        hipLaunchKernelGGL((k_xstress<T, NN, R>), dim3(blocks), dim3(kBlock), 0, s, (cx_t<T>*)spec, lpc, NS, phase,
                           (const T*)C21, t);
    })
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

// TX: columns per tile so that TX * (L / R) <= 256 and TX divides M.
static inline int col_tile(int L, int M)
{
    const int G = L / radix_col(L);
    int tx = kBlock / G;
    return tx < M ? tx : M;
}

template <typename T>
int launch_ypass(int dir, int n1, int n2, int n3, int ncomp, long NS, void* spec, const void* tw, hipStream_t s)
{
    const int M = n1 / 2;
    const int TX = col_tile(n2, M);
    const cx_t<T>* t = (const cx_t<T>*)tw;
    NM_SIZE_SWITCH(n2, {
        constexpr int R = NN >= 8 ? 8 : NN;
        constexpr int G = NN / R;
        dim3 grid(M / TX, n3, ncomp), block(TX * G);
        if (dir < 0)
            hipLaunchKernelGGL((k_ypass<T, NN, R, -1>), grid, block, 0, s, (cx_t<T>*)spec, (long)M, (long)n2 * M, NS,
                               TX, t);
        else
            hipLaunchKernelGGL((k_ypass<T, NN, R, +1>), grid, block, 0, s, (cx_t<T>*)spec, (long)M, (long)n2 * M, NS,
                               TX, t);
    })
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <typename T, int L>
static void zspec_dispatch(int op, dim3 grid, dim3 block, hipStream_t s, cx_t<T>* spec, long NS, int TX,
                           const SpecParams& sp, const cx_t<T>* t)
{
    constexpr int R = L >= 8 ? 8 : L;
    if (op == ZOP_GRAD) hipLaunchKernelGGL((k_zspec<T, L, R, ZOP_GRAD>), grid, block, 0, s, spec, NS, TX, sp, t);
    else if (op == ZOP_DIV) hipLaunchKernelGGL((k_zspec<T, L, R, ZOP_DIV>), grid, block, 0, s, spec, NS, TX, sp, t);
    else hipLaunchKernelGGL((k_zspec<T, L, R, ZOP_PRECOND>), grid, block, 0, s, spec, NS, TX, sp, t);
}

template <typename T> int launch_zspec(int op, const SpecParams& sp, long NS, void* spec, const void* tw, hipStream_t s)
{
    const int M = sp.n1 / 2;
    const cx_t<T>* t = (const cx_t<T>*)tw;
    cx_t<T>* d = (cx_t<T>*)spec;
    if (sp.n3 == 1) {
        const int TX = M < kBlock ? M : kBlock;
        zspec_dispatch<T, 1>(op, dim3(M / TX, sp.n2), dim3(TX), s, d, NS, TX, sp, t);
    } else {
        const int TX = col_tile(sp.n3, M);
        NM_SIZE_SWITCH(sp.n3, {
            constexpr int R = NN >= 8 ? 8 : NN;
            zspec_dispatch<T, NN>(op, dim3(M / TX, sp.n2), dim3(TX * (NN / R)), s, d, NS, TX, sp, t);
        })
    }
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

#define NM_INST(T)                                                                                                     \
    template int launch_xfwd<T>(int, int, const XFwdArgs&, const void*, hipStream_t);                                  \
    template int launch_xinv<T>(int, int, const XInvArgs&, const void*, hipStream_t);                                  \
    template int launch_xstress<T>(int, void*, long, long, const uint16_t*, const void*, const void*, hipStream_t);    \
    template int launch_ypass<T>(int, int, int, int, int, long, void*, const void*, hipStream_t);                      \
    template int launch_zspec<T>(int, const SpecParams&, long, void*, const void*, hipStream_t);
NM_INST(double)
NM_INST(float)

} // namespace nm
