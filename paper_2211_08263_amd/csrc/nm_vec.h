// Host launchers of the pointwise vector, reduction and Newmark kernels (nm_vec.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nm {

enum ReduceAction { RED_STORE_RR = 0, RED_ALPHA = 1, RED_RZ_INIT = 2, RED_BETA = 3, RED_STORE_SLOT = 4, RED_RR_CHECK = 5 };

// Deterministic sum of n per-block partials into the scalar block, then the action.
// x += alpha p, alpha read from the device (the deferred last update of a Krylov loop).
template <typename T> int launch_axpy_scal(T* x, const T* p, const double* alpha, long n, hipStream_t s);
// Arm a batched Krylov loop: clear S_STOP and S_ITER, set S_THR2, S_LIMIT, S_MODE (1: run
// exactly `limit` iterations).
int launch_loop_init(double* scal, double thr2, int limit, int fixed, hipStream_t s);
// guarded: the kernel does nothing once scal[S_STOP] is set.  RED_RR_CHECK stores r.r,
// counts the iteration and sets S_STOP when the loop is done (see ScalarSlot).
int launch_reduce(const double* partials, int n, double* scal, int action, int slot, hipStream_t s,
                  bool guarded = false);
// The same for nb independent Krylov loops run together (one block per loop): loop b sums
// partials [b n, (b + 1) n) into scal + b S_COUNT.  A loop whose S_STOP is set is frozen
// instead of skipped: RED_ALPHA and RED_BETA then store zero, so that its iterate receives the
// deferred last update once and then stays, and RED_RR_CHECK no longer counts.
int launch_reduce_multi(const double* partials, int n, int nb, double* scal, int action, hipStream_t s);

// Number of partials written by the grid-stride kernels below.
int vec_blocks(long n);

// r = b - q (masked entries -> 0), partial sums of r.r.
template <typename T>
int launch_residual(const T* b, const T* q, T* r, const uint8_t* mask, long N, int ncomp, double* partials,
                    hipStream_t s, float* r32 = nullptr);
// out = a + c * b.
template <typename T> int launch_axpby(T* out, const T* a, const T* b, double c, long n, hipStream_t s);
// y (FP32) = (float) x (FP64);  x64 += (double) d32
int launch_cast_d2f(float* y, const double* x, long n, hipStream_t s);
int launch_add_f2d(double* x, const float* d, long n, hipStream_t s);
// x += (double)(d + alpha[0] p): the last PCG update of an FP32 correction d folded into x.
int launch_add_f2d_axpy(double* x, const float* d, const float* p, const double* alpha, long n, hipStream_t s);
template <typename T> int launch_fill(T* x, T v, long n, hipStream_t s);
// r = P (b - q) for an FP32 q (FP64 arithmetic), partial sums of r.r.
int launch_residual_f32q(const double* b, const float* q, double* r, const uint8_t* mask, long N, double* partials,
                         hipStream_t s, float* r32 = nullptr);
// r <- P (r - q) in place for an FP32 q (FP64 arithmetic), partial sums of r.r.
int launch_update_f32q(double* r, const float* q, const uint8_t* mask, long N, double* partials, hipStream_t s,
                       float* r32 = nullptr);
// r = P (b - sum_c U3[c] G_c) with the three Gamma lifting responses G (3 x (3 x N)),
// partial sums of r.r (vec_blocks(3 N) of them).
int launch_lift_residual(const double* b, const double* G, const double* U3, const uint8_t* mask, long N, double* r,
                         double* partials, hipStream_t s, float* r32 = nullptr);
template <typename T> int launch_copy(T* dst, const T* src, long n, hipStream_t s);
// partial sums of a.b (FP64 accumulation)
template <typename T> int launch_dot(const T* a, const T* b, long n, double* partials, hipStream_t s);

// x[j*N + gidx[p]] = (per_point ? U[dim*p + j] : U[j]) for p < ng, j < dim
int launch_set_gamma(double* x, const int64_t* gidx, long ng, const double* U, int per_point, int dim, long N,
                     hipStream_t s);
int launch_set_gamma_f32(float* x, const int64_t* gidx, long ng, const double* U, int per_point, int dim, long N,
                         hipStream_t s);
// out[dim*p + j] = x[j*N + gidx[p]]
int launch_gather_gamma(double* out, const double* x, const int64_t* gidx, long ng, int dim, long N, hipStream_t s);

// Newmark predictor: ut = u + dt v + dt^2 (1/2 - beta) a ; b = rho(phase) ut, and with a
// viscous coefficient per phase (damp, or null) b -= beta dt^2 damp(phase) (v + (1 - gamma) dt a).
// rho is the operator density (rho + gamma dt damp with damping).
int launch_predictor(const double* u, const double* v, const double* a, double* ut, double* b,
                     const uint16_t* phase, const double* rho, const double* damp, long N, int ncomp, double dt,
                     double beta, double gam, hipStream_t s);
// Newmark corrector (an = (un - ut)/(beta dt^2); v += dt((1-g) a + g an); a = an) fused
// with the next predictor (ut = un + dt v + dt^2 (1/2 - beta) a) and b = rho ut (damping as in
// launch_predictor, with the new v and a).
// inc (or null): corrector_blocks(N) per-block sums of |ut_new - un|^2; feat (or null):
// unscaled BF16 state features [N][16] of the new state (u, dt v, dt^2 (1/2 - beta) a).
int corrector_blocks(long N);
int launch_corrector_predictor(const double* un, double* ut, double* v, double* a, double* b, const uint16_t* phase,
                               const double* rho, const double* damp, long N, int ncomp, double dt, double beta,
                               double gam, double* inc, uint16_t* feat, hipStream_t s);
// Initial acceleration from q = A u0: a0 = (rho u0 - q) / (beta dt^2 rho) = div(C : grad^s u0) / rho
int launch_accel0(double* a, const double* u0, const double* q, const uint16_t* phase, const double* rho, long N,
                  int ncomp, double bdt2, hipStream_t s);
// Initial acceleration with viscous damping: a0 = (q - damp(phase) v0) / rho(phase), q = div(C :
// grad^s u0) (null for u0 = 0), rho the true density.
int launch_accel0_damped(double* a, const double* q, const double* v, const uint16_t* phase, const double* rho,
                         const double* damp, long N, int ncomp, hipStream_t s);
// Explicit central-difference scheme, Gamma voxels after the velocity pass: with vb = v there,
// f = 2 rho / dt (Udot - vb), v = Udot, a += f / rho, F[dim*p + j] = f (eq.
// Explicit_linear_momentum_arranged_3D and the force that prescribes the velocity).
// Udot: dim values (uniform) or dim*ng values (per point).
int launch_explicit_gamma(double* v, double* a, const uint16_t* phase, const double* rho, const int64_t* gidx, long ng,
                          const double* Udot, int per_point, int dim, long N, double dt, double* F, hipStream_t s);
// Partial sums of sum rho(phase) x^2 over a 3 x N field (vec_blocks(3 N) of them).
int launch_rho_norm2(const double* x, const uint16_t* phase, const double* rho, long N, double* partials,
                     hipStream_t s);
// x = y / rho(phase) for 3 x N fields.
int launch_div_rho(double* x, const double* y, const uint16_t* phase, const double* rho, long N, hipStream_t s);
// Second-order Taylor start: x = u + dt v + dt^2/2 a
int launch_taylor(double* x, const double* u, const double* v, const double* a, long n, double dt, hipStream_t s);

} // namespace nm
