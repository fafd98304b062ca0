// Pointwise vector, reduction and Newmark kernels (grid-stride, coalesced SoA).
#include "nm_common.h"
#include "nm_passes.h"
#include "nm_vec.h"

namespace nm {

constexpr int kVecBlocksMax = 2048;

int vec_blocks(long n)
{
    long b = (n + kBlock * 4 - 1) / (kBlock * 4);
    if (b < 1) b = 1;
    return (int)(b < kVecBlocksMax ? b : kVecBlocksMax);
}

__device__ __forceinline__ double wave_sum_v(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double block_sum_v(double v)
{
    __shared__ double sh[16];
    v = wave_sum_v(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x + 63) / 64; i++) s += sh[i];
    return s;
}

// One block of 1024 threads: thread i sums partials i, i+1024, ... in order.
__global__ __launch_bounds__(1024) void k_reduce(const double* __restrict__ part, int n, double* scal, int action,
                                                 int slot, int guarded)
{
    if (guarded && scal[S_STOP] != 0.0) return;
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) v += part[i];
    const double s = block_sum_v(v);
    if (threadIdx.x == 0) {
        switch (action) {
        case RED_STORE_RR: scal[S_RR] = s; break;
        case RED_RR_CHECK: {
            scal[S_RR] = s;
            const double it = scal[S_ITER] + 1.0;
            scal[S_ITER] = it;
            const bool done = scal[S_MODE] != 0.0 ? it >= scal[S_LIMIT]
                                                  : (s <= scal[S_THR2] || it >= scal[S_LIMIT] || !(s < 1e300));
            if (done) scal[S_STOP] = 1.0;
            break;
        }
        case RED_ALPHA:
            scal[S_PQ] = s;
            scal[S_ALPHA] = scal[S_RZ] / s;
            break;
        case RED_RZ_INIT:
            scal[S_RZ] = s;
            scal[S_FIRST] = 1.0;
            break;
        case RED_BETA:
            scal[S_BETA] = s / scal[S_RZ];
            scal[S_RZ] = s;
            scal[S_FIRST] = 0.0;
            break;
        default: scal[slot] = s; break;
        }
    }
}

__global__ __launch_bounds__(1024) void k_reduce_multi(const double* __restrict__ part, int n, double* scal_all,
                                                       int action)
{
    const double* pb = part + (long)blockIdx.x * n;
    double* scal = scal_all + (long)blockIdx.x * S_COUNT;
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) v += pb[i];
    const double s = block_sum_v(v);
    if (threadIdx.x == 0) {
        const bool frozen = scal[S_STOP] != 0.0;
        switch (action) {
        case RED_RR_CHECK: {
            if (frozen) break;
            scal[S_RR] = s;
            const double it = scal[S_ITER] + 1.0;
            scal[S_ITER] = it;
            if (s <= scal[S_THR2] || it >= scal[S_LIMIT] || !(s < 1e300)) scal[S_STOP] = 1.0;
            break;
        }
        case RED_ALPHA:
            scal[S_PQ] = s;
            scal[S_ALPHA] = frozen ? 0.0 : scal[S_RZ] / s;
            break;
        case RED_RZ_INIT:
            scal[S_RZ] = s;
            scal[S_FIRST] = 1.0;
            break;
        case RED_BETA:
            scal[S_BETA] = frozen ? 0.0 : s / scal[S_RZ];
            scal[S_RZ] = s;
            scal[S_FIRST] = 0.0;
            break;
        default: scal[S_RR] = s; break;
        }
    }
}
int launch_reduce_multi(const double* partials, int n, int nb, double* scal, int action, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_multi, dim3(nb), dim3(1024), 0, s, partials, n, scal, action);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

// x += alpha p with alpha read from the device
template <typename T>
__global__ __launch_bounds__(kBlock) void k_axpy_scal(T* __restrict__ x, const T* __restrict__ p,
                                                      const double* __restrict__ alpha, long n)
{
    const T a = (T)alpha[0];
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        x[i] = x[i] + a * p[i];
}
template <typename T> int launch_axpy_scal(T* x, const T* p, const double* alpha, long n, hipStream_t s)
{
    hipLaunchKernelGGL((k_axpy_scal<T>), dim3(vec_blocks(n)), dim3(kBlock), 0, s, x, p, alpha, n);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}
template int launch_axpy_scal<double>(double*, const double*, const double*, long, hipStream_t);
template int launch_axpy_scal<float>(float*, const float*, const double*, long, hipStream_t);

__global__ void k_loop_init(double* scal, double thr2, double limit, double mode)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        scal[S_STOP] = 0.0;
        scal[S_ITER] = 0.0;
        scal[S_THR2] = thr2;
        scal[S_LIMIT] = limit;
        scal[S_MODE] = mode;
    }
}
int launch_loop_init(double* scal, double thr2, int limit, int fixed, hipStream_t s)
{
    hipLaunchKernelGGL(k_loop_init, dim3(1), dim3(64), 0, s, scal, thr2, (double)limit, (double)fixed);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

int launch_reduce(const double* partials, int n, double* scal, int action, int slot, hipStream_t s, bool guarded)
{
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, s, partials, n, scal, action, slot, guarded ? 1 : 0);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_residual(const T* __restrict__ b, const T* __restrict__ q, T* __restrict__ r,
                                                     const uint8_t* __restrict__ mask, long N, long n,
                                                     double* partials, float* __restrict__ r32)
{
    double acc = 0.0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        T v = b[i] - q[i];
        if (mask && mask[i % N]) v = 0;
        r[i] = v;
        if (r32) r32[i] = (float)v;
        acc += (double)v * (double)v;
    }
    const double s = block_sum_v(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

template <typename T>
int launch_residual(const T* b, const T* q, T* r, const uint8_t* mask, long N, int ncomp, double* partials,
                    hipStream_t s, float* r32)
{
    const long n = N * ncomp;
    hipLaunchKernelGGL((k_residual<T>), dim3(vec_blocks(n)), dim3(kBlock), 0, s, b, q, r, mask, N, n, partials, r32);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

// r = P (b - q) with an FP32 q, accumulated in FP64; partial sums of r.r.
__global__ __launch_bounds__(kBlock) void k_residual_f32q(const double* __restrict__ b, const float* __restrict__ q,
                                                          double* __restrict__ r, const uint8_t* __restrict__ mask,
                                                          long N, long n, double* partials, float* __restrict__ r32)
{
    double acc = 0.0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        double v = b[i] - (double)q[i];
        if (mask && mask[i % N]) v = 0;
        r[i] = v;
        if (r32) r32[i] = (float)v;
        acc += v * v;
    }
    const double s = block_sum_v(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}
int launch_residual_f32q(const double* b, const float* q, double* r, const uint8_t* mask, long N, double* partials,
                         hipStream_t s, float* r32)
{
    const long n = 3 * N;
    hipLaunchKernelGGL(k_residual_f32q, dim3(vec_blocks(n)), dim3(kBlock), 0, s, b, q, r, mask, N, n, partials, r32);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

// r <- P (r - q) in place for an FP32 q (FP64 arithmetic); partial sums of r.r.
__global__ __launch_bounds__(kBlock) void k_update_f32q(double* r, const float* __restrict__ q,
                                                        const uint8_t* __restrict__ mask, long N, long n,
                                                        double* partials, float* __restrict__ r32)
{
    double acc = 0.0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        double v = r[i] - (double)q[i];
        if (mask && mask[i % N]) v = 0;
        r[i] = v;
        if (r32) r32[i] = (float)v;
        acc += v * v;
    }
    const double s = block_sum_v(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}
int launch_update_f32q(double* r, const float* q, const uint8_t* mask, long N, double* partials, hipStream_t s,
                       float* r32)
{
    const long n = 3 * N;
    hipLaunchKernelGGL(k_update_f32q, dim3(vec_blocks(n)), dim3(kBlock), 0, s, r, q, mask, N, n, partials, r32);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

// r = P (b - (U0 G0 + U1 G1 + U2 G2)), G_c: 3 x N fields stored one after another;
// partial sums of r.r.
__global__ __launch_bounds__(kBlock) void k_lift_residual(const double* __restrict__ b, const double* __restrict__ G,
                                                          double U0, double U1, double U2,
                                                          const uint8_t* __restrict__ mask, long N, long n,
                                                          double* __restrict__ r, double* partials,
                                                          float* __restrict__ r32)
{
    double acc = 0.0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        // components with a zero prescribed value are skipped (their responses are not read)
        double q = U0 != 0.0 ? U0 * G[i] : 0.0;
        if (U1 != 0.0) q += U1 * G[n + i];
        if (U2 != 0.0) q += U2 * G[2 * n + i];
        double v = b[i] - q;
        if (mask[i % N]) v = 0;
        r[i] = v;
        if (r32) r32[i] = (float)v;
        acc += v * v;
    }
    const double s = block_sum_v(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}
int launch_lift_residual(const double* b, const double* G, const double* U3, const uint8_t* mask, long N, double* r,
                         double* partials, hipStream_t s, float* r32)
{
    const long n = 3 * N;
    hipLaunchKernelGGL(k_lift_residual, dim3(vec_blocks(n)), dim3(kBlock), 0, s, b, G, U3[0], U3[1], U3[2], mask, N, n,
                       r, partials, r32);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_axpby(T* out, const T* a, const T* b, double c, long n)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        out[i] = a[i] + (T)c * b[i];
}
template <typename T> int launch_axpby(T* out, const T* a, const T* b, double c, long n, hipStream_t s)
{
    hipLaunchKernelGGL((k_axpby<T>), dim3(vec_blocks(n)), dim3(kBlock), 0, s, out, a, b, c, n);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

__global__ __launch_bounds__(kBlock) void k_cast_d2f(float* y, const double* x, long n)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        y[i] = (float)x[i];
}
int launch_cast_d2f(float* y, const double* x, long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_cast_d2f, dim3(vec_blocks(n)), dim3(kBlock), 0, s, y, x, n);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

__global__ __launch_bounds__(kBlock) void k_add_f2d(double* x, const float* d, long n)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        x[i] += (double)d[i];
}
int launch_add_f2d(double* x, const float* d, long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_add_f2d, dim3(vec_blocks(n)), dim3(kBlock), 0, s, x, d, n);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

// x += (double)(d + alpha p) with the FP32 sum rounded as the separate update would round it
__global__ __launch_bounds__(kBlock) void k_add_f2d_axpy(double* x, const float* __restrict__ d,
                                                         const float* __restrict__ p, const double* __restrict__ alpha,
                                                         long n)
{
    const float a = (float)alpha[0];
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const float di = d[i] + a * p[i];
        x[i] += (double)di;
    }
}
int launch_add_f2d_axpy(double* x, const float* d, const float* p, const double* alpha, long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_add_f2d_axpy, dim3(vec_blocks(n)), dim3(kBlock), 0, s, x, d, p, alpha, n);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <typename T> __global__ __launch_bounds__(kBlock) void k_fill(T* x, T v, long n)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) x[i] = v;
}
template <typename T> int launch_fill(T* x, T v, long n, hipStream_t s)
{
    hipLaunchKernelGGL((k_fill<T>), dim3(vec_blocks(n)), dim3(kBlock), 0, s, x, v, n);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <typename T> __global__ __launch_bounds__(kBlock) void k_copy(T* d, const T* s, long n)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) d[i] = s[i];
}
template <typename T> int launch_copy(T* dst, const T* src, long n, hipStream_t s)
{
    hipLaunchKernelGGL((k_copy<T>), dim3(vec_blocks(n)), dim3(kBlock), 0, s, dst, src, n);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_dot(const T* __restrict__ a, const T* __restrict__ b, long n,
                                                double* partials)
{
    double acc = 0.0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        acc += (double)a[i] * (double)b[i];
    const double s = block_sum_v(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}
template <typename T> int launch_dot(const T* a, const T* b, long n, double* partials, hipStream_t s)
{
    hipLaunchKernelGGL((k_dot<T>), dim3(vec_blocks(n)), dim3(kBlock), 0, s, a, b, n, partials);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <typename T>
__global__ void k_set_gamma(T* x, const int64_t* gidx, long ng, const double* U, int per_point, int dim, long N)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ng * dim) return;
    const long p = i / dim;
    const int j = (int)(i % dim);
    x[j * N + gidx[p]] = (T)(per_point ? U[i] : U[j]);
}
template <typename T>
static int set_gamma_impl(T* x, const int64_t* gidx, long ng, const double* U, int per_point, int dim, long N,
                          hipStream_t s)
{
    if (ng == 0) return 0;
    const long n = ng * dim;
    hipLaunchKernelGGL(k_set_gamma<T>, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, x, gidx, ng,
                       U, per_point, dim, N);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}
int launch_set_gamma(double* x, const int64_t* gidx, long ng, const double* U, int per_point, int dim, long N,
                     hipStream_t s)
{
    return set_gamma_impl<double>(x, gidx, ng, U, per_point, dim, N, s);
}
int launch_set_gamma_f32(float* x, const int64_t* gidx, long ng, const double* U, int per_point, int dim, long N,
                         hipStream_t s)
{
    return set_gamma_impl<float>(x, gidx, ng, U, per_point, dim, N, s);
}

__global__ void k_gather_gamma(double* out, const double* x, const int64_t* gidx, long ng, int dim, long N)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ng * dim) return;
    const long p = i / dim;
    const int j = (int)(i % dim);
    out[i] = x[j * N + gidx[p]];
}
int launch_gather_gamma(double* out, const double* x, const int64_t* gidx, long ng, int dim, long N, hipStream_t s)
{
    if (ng == 0) return 0;
    const long n = ng * dim;
    hipLaunchKernelGGL(k_gather_gamma, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, out, x, gidx,
                       ng, dim, N);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

__global__ __launch_bounds__(kBlock) void k_predictor(const double* __restrict__ u, const double* __restrict__ v,
                                                      const double* __restrict__ a, double* __restrict__ ut,
                                                      double* __restrict__ b, const uint16_t* __restrict__ phase,
                                                      const double* __restrict__ rho, const double* __restrict__ damp,
                                                      long N, long n, double dt, double c2, double bdt2, double gdt1)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const double w = u[i] + dt * v[i] + c2 * a[i];
        const int g = phase[i % N];
        ut[i] = w;
        double bi = rho[g] * w;
        if (damp) bi -= bdt2 * damp[g] * (v[i] + gdt1 * a[i]);
        b[i] = bi;
    }
}
int launch_predictor(const double* u, const double* v, const double* a, double* ut, double* b, const uint16_t* phase,
                     const double* rho, const double* damp, long N, int ncomp, double dt, double beta, double gam,
                     hipStream_t s)
{
    const long n = N * ncomp;
    hipLaunchKernelGGL(k_predictor, dim3(vec_blocks(n)), dim3(kBlock), 0, s, u, v, a, ut, b, phase, rho, damp, N, n,
                       dt, dt * dt * (0.5 - beta), beta * dt * dt, (1.0 - gam) * dt);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

// BF16 (round to nearest even) of a float, for the feature output of the corrector.
__device__ __forceinline__ uint16_t bf16_rne(float f)
{
    uint32_t x = __float_as_uint(f);
    if ((x & 0x7f800000u) == 0x7f800000u) return (uint16_t)(x >> 16); // inf / nan
    x += 0x7fffu + ((x >> 16) & 1u);
    return (uint16_t)(x >> 16);
}

// Corrector of this step fused with the predictor of the next one:
// a_n = (u_n - u~)/(beta dt^2), v_n = v + dt((1 - gamma) a + gamma a_n), then
// u~' = u_n + dt v_n + dt^2 (1/2 - beta) a_n and b' = rho u~' (ut and b overwritten; with
// damping b' = rho u~' - beta dt^2 c (v_n + (1 - gamma) dt a_n), rho the operator density).
// inc (or null): per-block sums of |u~' - u_n|^2 (the learned start's scale).
// feat (or null): the learned start's state features of the new state, unscaled, BF16
// [N][16]: (u_n, dt v_n, dt^2 (1/2 - beta) a_n) per component, channels 9..15 zero.
// One thread per voxel and its three components.
__global__ __launch_bounds__(kBlock) void k_corrector_predictor(const double* __restrict__ un, double* __restrict__ ut,
                                                                double* __restrict__ v, double* __restrict__ a,
                                                                double* __restrict__ b,
                                                                const uint16_t* __restrict__ phase,
                                                                const double* __restrict__ rho,
                                                                const double* __restrict__ damp, long N,
                                                                double dt, double inv_bdt2, double gam, double c2,
                                                                double bdt2, double gdt1,
                                                                double* __restrict__ inc, uint16_t* __restrict__ feat)
{
    double acc = 0.0;
    for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < N; p += (long)gridDim.x * blockDim.x) {
        const int g = phase[p];
        const double rp = rho[g];
        const double cb = damp ? bdt2 * damp[g] : 0.0;
        uint16_t f[16];
#pragma unroll
        for (int k = 0; k < 16; k++) f[k] = 0;
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const long i = c * N + p;
            const double u = un[i];
            const double an = (u - ut[i]) * inv_bdt2;
            const double vn = v[i] + dt * ((1.0 - gam) * a[i] + gam * an);
            v[i] = vn;
            a[i] = an;
            const double w = u + dt * vn + c2 * an;
            ut[i] = w;
            double bi = rp * w;
            if (damp) bi -= cb * (vn + gdt1 * an);
            b[i] = bi;
            acc += (w - u) * (w - u);
            f[c] = bf16_rne((float)u);
            f[3 + c] = bf16_rne((float)(dt * vn));
            f[6 + c] = bf16_rne((float)(c2 * an));
        }
        if (feat) {
#pragma unroll
            for (int k = 0; k < 16; k += 4) {
                const uint64_t wv = (uint64_t)f[k] | ((uint64_t)f[k + 1] << 16) | ((uint64_t)f[k + 2] << 32) |
                                    ((uint64_t)f[k + 3] << 48);
                *(uint64_t*)(feat + p * 16 + k) = wv;
            }
        }
    }
    if (inc) {
        __shared__ double sh[kBlock / 64];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
#pragma unroll
            for (int w = 0; w < kBlock / 64; w++) t += sh[w];
            inc[blockIdx.x] = t;
        }
    }
}
int corrector_blocks(long N) { return vec_blocks(N); }
int launch_corrector_predictor(const double* un, double* ut, double* v, double* a, double* b, const uint16_t* phase,
                               const double* rho, const double* damp, long N, int ncomp, double dt, double beta,
                               double gam, double* inc, uint16_t* feat, hipStream_t s)
{
    if (ncomp != 3) return -1;
    hipLaunchKernelGGL(k_corrector_predictor, dim3(corrector_blocks(N)), dim3(kBlock), 0, s, un, ut, v, a, b, phase,
                       rho, damp, N, dt, 1.0 / (beta * dt * dt), gam, dt * dt * (0.5 - beta), beta * dt * dt,
                       (1.0 - gam) * dt, inc, feat);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}


__global__ __launch_bounds__(kBlock) void k_accel0(double* a, const double* u0, const double* q,
                                                   const uint16_t* phase, const double* rho, long N, long n,
                                                   double bdt2)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const double r = rho[phase[i % N]];
        a[i] = (r * u0[i] - q[i]) / (bdt2 * r);
    }
}
int launch_accel0(double* a, const double* u0, const double* q, const uint16_t* phase, const double* rho, long N,
                  int ncomp, double bdt2, hipStream_t s)
{
    const long n = N * ncomp;
    hipLaunchKernelGGL(k_accel0, dim3(vec_blocks(n)), dim3(kBlock), 0, s, a, u0, q, phase, rho, N, n, bdt2);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

__global__ __launch_bounds__(kBlock) void k_accel0_damped(double* a, const double* q, const double* v,
                                                          const uint16_t* phase, const double* rho,
                                                          const double* damp, long N, long n)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const int g = phase[i % N];
        a[i] = ((q ? q[i] : 0.0) - damp[g] * v[i]) / rho[g];
    }
}
int launch_accel0_damped(double* a, const double* q, const double* v, const uint16_t* phase, const double* rho,
                         const double* damp, long N, int ncomp, hipStream_t s)
{
    const long n = N * ncomp;
    hipLaunchKernelGGL(k_accel0_damped, dim3(vec_blocks(n)), dim3(kBlock), 0, s, a, q, v, phase, rho, damp, N, n);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

__global__ __launch_bounds__(kBlock) void k_explicit_gamma(double* __restrict__ v, double* __restrict__ a,
                                                          const uint16_t* __restrict__ phase,
                                                          const double* __restrict__ rho,
                                                          const int64_t* __restrict__ gidx, long ng,
                                                          const double* __restrict__ Udot, int per_point, int dim,
                                                          long N, double dt, double* __restrict__ F)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ng * dim) return;
    const long p = e / dim;
    const int j = (int)(e % dim);
    const long g = gidx[p];
    const long i = j * N + g;
    const double r = rho[phase[g]];
    const double U = per_point ? Udot[dim * p + j] : Udot[j];
    const double f = 2.0 * r / dt * (U - v[i]);
    v[i] = U;
    a[i] = a[i] + f / r;
    F[dim * p + j] = f;
}
int launch_explicit_gamma(double* v, double* a, const uint16_t* phase, const double* rho, const int64_t* gidx, long ng,
                          const double* Udot, int per_point, int dim, long N, double dt, double* F, hipStream_t s)
{
    const long n = ng * dim;
    if (n == 0) return 0;
    hipLaunchKernelGGL(k_explicit_gamma, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, v, a, phase,
                       rho, gidx, ng, Udot, per_point, dim, N, dt, F);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

__global__ __launch_bounds__(kBlock) void k_rho_norm2(const double* __restrict__ x, const uint16_t* __restrict__ phase,
                                                     const double* __restrict__ rho, long N, long n,
                                                     double* __restrict__ partials)
{
    double acc = 0.0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        acc += rho[phase[i % N]] * x[i] * x[i];
    const double s = block_sum_v(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}
int launch_rho_norm2(const double* x, const uint16_t* phase, const double* rho, long N, double* partials,
                     hipStream_t s)
{
    const long n = 3 * N;
    hipLaunchKernelGGL(k_rho_norm2, dim3(vec_blocks(n)), dim3(kBlock), 0, s, x, phase, rho, N, n, partials);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

__global__ __launch_bounds__(kBlock) void k_div_rho(double* __restrict__ x, const double* __restrict__ y,
                                                   const uint16_t* __restrict__ phase, const double* __restrict__ rho,
                                                   long N, long n)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        x[i] = y[i] / rho[phase[i % N]];
}
int launch_div_rho(double* x, const double* y, const uint16_t* phase, const double* rho, long N, hipStream_t s)
{
    const long n = 3 * N;
    hipLaunchKernelGGL(k_div_rho, dim3(vec_blocks(n)), dim3(kBlock), 0, s, x, y, phase, rho, N, n);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

__global__ __launch_bounds__(kBlock) void k_taylor(double* x, const double* u, const double* v, const double* a, long n,
                                                   double dt)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        x[i] = u[i] + dt * v[i] + 0.5 * dt * dt * a[i];
}
int launch_taylor(double* x, const double* u, const double* v, const double* a, long n, double dt, hipStream_t s)
{
    hipLaunchKernelGGL(k_taylor, dim3(vec_blocks(n)), dim3(kBlock), 0, s, x, u, v, a, n, dt);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

template int launch_residual<double>(const double*, const double*, double*, const uint8_t*, long, int, double*,
                                     hipStream_t, float*);
template int launch_residual<float>(const float*, const float*, float*, const uint8_t*, long, int, double*,
                                    hipStream_t, float*);
template int launch_axpby<double>(double*, const double*, const double*, double, long, hipStream_t);
template int launch_axpby<float>(float*, const float*, const float*, double, long, hipStream_t);
template int launch_fill<double>(double*, double, long, hipStream_t);
template int launch_fill<float>(float*, float, long, hipStream_t);
template int launch_fill<int>(int*, int, long, hipStream_t);
template int launch_copy<double>(double*, const double*, long, hipStream_t);
template int launch_copy<float>(float*, const float*, long, hipStream_t);
template int launch_dot<double>(const double*, const double*, long, double*, hipStream_t);
template int launch_dot<float>(const float*, const float*, long, double*, hipStream_t);

} // namespace nm
