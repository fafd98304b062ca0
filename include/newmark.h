/*
 * newmark.h -- C ABI of the MI355X (gfx950) implicit FFT Newmark solver.
 *
 * Implements the hot path of Sancho, Rey de Pedraza, Lafourcade, Lebensohn
 * and Segurado, "An implicit FFT-based method for wave propagation in elastic
 * heterogeneous media" (arXiv 2211.08263): each Newmark-beta step (eq. Newmark,
 * beta = 1/4, gamma = 1/2) solves the discretized momentum balance of eq.
 * (ND_consv_lm_Newmark_ord) with the matrix-free operator of eq.
 * (Fourier_ND_A), preconditioned conjugate gradients (section 2.2.3) and the
 * reference-medium preconditioner of eqs. (precond)-(acous), while the
 * displacement is prescribed on the voxel set Gamma (eqs. (f), (new)).
 *
 * Conventions
 *  - Grid n1 x n2 x n3 voxels, x fastest; voxel (i,j,k) has linear index
 *    i + n1*(j + n2*k) and centre ((i+1/2) L1/n1, ...) (section 2.2.3).
 *  - Vector fields are SoA: component c of voxel v at c*N + v, N = n1 n2 n3.
 *    Device fields always hold 3 components; for dim == 2 (plane strain,
 *    n3 == 1) the third component is kept at zero.
 *  - Stiffness: per phase, the 21 upper-triangle entries (row major) of the
 *    6x6 Voigt matrix in the order 11,22,33,23,13,12 with engineering shear
 *    strains.  Density: one value per phase.
 *  - Discrete frequencies in standard DFT order with the Nyquist bin set to
 *    zero (the paper uses odd grids only; this keeps the operator real,
 *    symmetric and positive definite on even grids).
 *  - Every function returns NM_OK (0) or a negative NM_E* code; the message is
 *    available from nm_last_error().  No exception crosses the ABI.
 *  - One context per host thread.  All device work runs on the context's HIP
 *    stream.
 */
#ifndef NEWMARK_H
#define NEWMARK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum nm_status {
    NM_OK = 0,
    NM_EINVAL = -1,       /* bad argument: shapes, dtypes, Gamma index range, null pointers */
    NM_EUNSUPPORTED = -2, /* dim not 2/3, or an axis not a power of two in [8, 512] (n3 == 1 in 2D) */
    NM_ENOMEM = -3,       /* device or pinned-host allocation failed */
    NM_ENOTCONV = -4,     /* Krylov solve hit max_iter; the state is left at the previous step */
    NM_ESINGULAR = -5,    /* zero pivot in the Green-matrix factorization */
    NM_ENAN = -6,         /* non-finite value in the prescribed displacement or a residual */
    NM_EHIP = -7          /* HIP runtime error */
};

enum nm_dtype { NM_FP64 = 0, NM_FP32 = 1 };
enum nm_precision { NM_PREC_FP64 = 0, NM_PREC_MIXED = 1 };
enum nm_route { NM_ROUTE_AUTO = 0, NM_ROUTE_GREEN = 1, NM_ROUTE_PROJECTED = 2 };
enum nm_warm_start { NM_WS_COLD = 0, NM_WS_PREV = 1, NM_WS_TAYLOR = 2, NM_WS_LEARNED = 3 };
/* Differentiation rules: the symbol of D_k in eq. Fourier_ND_A, the preconditioner of eq. precond
 * and both time steppers.  SPECTRAL: i xi_k (the paper's; Nyquist bin zero).  CENTRED2: the
 * centred difference (f(x+h) - f(x-h))/(2h), symbol i sin(xi_k h)/h.  CENTRED4: the fourth-order
 * centred difference (-f(x+2h) + 8 f(x+h) - 8 f(x-h) + f(x-2h))/(12h), symbol
 * i (8 sin(xi_k h) - sin(2 xi_k h))/(6h).  h = L_k / n_k. */
enum nm_diff_rule { NM_DIFF_SPECTRAL = 0, NM_DIFF_CENTRED2 = 1, NM_DIFF_CENTRED4 = 2 };

/* Inputs of the paper's Algorithm 2 (KwData): microstructure, Gamma, initial
 * state, time increment and Newmark constants.  Host arrays are copied by
 * nm_newmark_init; the caller keeps ownership. */
typedef struct nm_problem {
    int dim;                  /* 2 (plane strain, n[2] == 1) or 3 */
    int n[3];                 /* voxels per axis */
    double L[3];              /* box lengths (L[2] ignored in 2D) */
    int n_phases;             /* >= 1, <= 65536 */
    const uint16_t* phase_id; /* host, N entries, each < n_phases */
    const double* C_voigt;    /* host, n_phases x 21 */
    const double* rho;        /* host, n_phases, > 0 */
    const int64_t* gamma_idx; /* host, n_gamma sorted unique voxel indices in [0, N) (may be NULL if n_gamma == 0) */
    int64_t n_gamma;
    const double* u0;         /* host, dim x N initial displacement, or NULL for zero */
    const double* v0;         /* host, dim x N initial velocity, or NULL for zero */
    double dt;                /* time increment */
    double beta;              /* Newmark beta (0.25) */
    double gamma_nm;          /* Newmark gamma (0.5) */
    const double* damping;    /* host, n_phases viscous coefficients c >= 0 per unit volume, or NULL:
                                 M a + C v + K u = f with C = diag(c(phase)) (section 5's viscous
                                 buffer against the second wave of periodic boxes), integrated by
                                 the same Newmark rule: the operator's density becomes
                                 rho + gamma dt c and the right-hand side
                                 (rho + gamma dt c) u~ - beta dt^2 c (v + (1 - gamma) dt a).
                                 Implicit scheme only (NM_EUNSUPPORTED with beta == 0 and any
                                 c > 0); all zeros is the undamped problem */
    int diff_rule;            /* nm_diff_rule: the derivative's Fourier symbol (section 5 suggests discrete
                                 finite-difference rules against the noise of large contrast) */
} nm_problem;

typedef struct nm_options {
    int precision;            /* nm_precision */
    int route;                /* nm_route: GREEN (paper, G matrix + LU) or PROJECTED (PCG on the free dofs) */
    double tol;               /* relative residual tolerance of each solve */
    int max_iter;             /* per solve (per inner solve in mixed precision) */
    double inner_tol;         /* mixed precision: smallest relative tolerance asked of an FP32 inner
                                 solve (each solve reduces its residual by max(inner_tol, half the
                                 factor the outer tolerance still needs)); <= 0 means 1e-5 */
    int max_sweeps;           /* mixed precision: maximum refinement sweeps per step */
    int warm_start;           /* nm_warm_start */
    double green_tol;         /* tolerance of the unit-force solves that build G */
    int compute_reaction;     /* projected route: also compute F on Gamma (one extra operator apply) */
    int true_residual;        /* projected route: report the FP64 ||P(b - A u)|| / ||b_ref|| of the solution
                                 (one extra FP64 operator apply) instead of the solver's own estimate */
    const double* green_in;   /* GREEN route: a stored Green matrix ((dim n_gamma)^2, row major, as
                                 nm_green_matrix returns it for this problem and dt) to reuse instead of
                                 the unit-force solves (section 3.2: the preprocessing of an RVE can be
                                 stored and reused), or NULL; host, copied */
    void (*green_progress)(int64_t done, int64_t total, void* user); /* GREEN route: called after each
                                 unit-force solve of nm_newmark_init, or each group solved together
                                 (may be NULL) */
    void* green_progress_user;
    int green_batch;          /* GREEN route: unit-force solves run together through one chain of kernels,
                                 in the context's precision (FP64: each column bit for bit the one a
                                 single solve gives): 0 picks the number from the grid (about 8M voxels of
                                 work, at most 16), 1 solves one at a time, k >= 2 solves k at a time (at
                                 most 64) */
} nm_options;

typedef struct nm_step_stats {
    int iters[2];             /* FP64 solves: PCG iterations (Green route: u_b, u_f; projected: [0], [1] = 0) */
    int sweeps;               /* mixed precision: FP64 refinement sweeps (Green route: of both solves) */
    int inner_iters;          /* mixed precision: total FP32 PCG iterations (Green route: of both solves) */
    double relres;            /* final relative residual: the FP64 residual of the solution when
                                 true_residual is set, else the value the stopping test used (the
                                 recursive residual; in mixed precision the last FP64 residual or
                                 a small final correction's recursive residual) */
    double relres0;           /* relative residual of the initial guess (first solve) */
    double t_step_ms;         /* wall time of the step (host clock, after a stream synchronize) */
    double t_warm_ms;         /* device time of the warm-start prediction (events on the stream) */
} nm_step_stats;

typedef struct nm_ctx nm_ctx;

/* Build the solver (beta > 0: the implicit Newmark method; beta == 0: the explicit
 * central-difference scheme, see nm_explicit_step): copies the problem to the device, forms the reference
 * medium (volume averages of C and rho, eq. (precond)), the FFT twiddle
 * tables, the Gamma route (GREEN: d*n_gamma unit-force solves of eq.
 * (solve_green) in the context's precision, or a stored G from options->green_in,
 * the matrix G of eq. (G) on the device and its LU factors with partial pivoting, also
 * on the device) and the initial acceleration a0 = (div(C : grad^s u0) - c v0) / rho
 * (c = 0 without damping).  hip_stream
 * may be NULL (a stream is created).  On success *out owns all resources. */
int nm_newmark_init(const nm_problem* pb, const nm_options* op, void* hip_stream, nm_ctx** out);

/* Advance one step: t_n = t_{n-1} + dt.  U_n (host) holds the prescribed
 * displacement, dim values (uniform on Gamma) when per_point == 0, or
 * dim*n_gamma values (point major) otherwise.  Returns after the stream has
 * synchronized.  On error the state stays at step n-1.  st may be NULL. */
int nm_newmark_step(nm_ctx* ctx, const double* U_n, int per_point, nm_step_stats* st);

/* The explicit central-difference scheme of section 2.3 (a context created with
 * pb->beta == 0 and pb->gamma_nm == 0.5; FP64; route AUTO or PROJECTED).  Each step
 * (eq. Central_diff_rule with eqs. b_explicit and Explicit_linear_momentum_arranged_3D):
 *     u_n  = u_{n-1} + dt v_{n-1} + dt^2/2 a_{n-1}
 *     v_b  = v_{n-1} + dt/2 a_{n-1} + dt/(2 rho) div(C : grad^s u_n)
 *     f_n  = 2 rho / dt (Udot_n - v_b) on Gamma, 0 elsewhere
 *     v_n  = v_b + dt/(2 rho) f_n    (so v_n = Udot_n on Gamma)
 *     a_n  = (div(C : grad^s u_n) + f_n) / rho
 * The velocity, not the displacement, is prescribed on Gamma.  Runs n_steps steps on the
 * context stream and synchronizes once.  Udot (host) holds n_steps rows of dim values
 * (uniform on Gamma, per_point == 0) or dim*n_gamma values (point major); row k is
 * Udot(t_{n+k+1}).  nm_get_state's F_gamma is f of the last step.  The scheme is stable
 * for dt <= 2 / omega_max (eq. Courant_stable; nm_omega2_max estimates omega_max^2); the
 * library does not check dt.  st (may be NULL) receives the mean wall time per step.
 * NM_EINVAL on a context of the implicit scheme or n_steps < 1; NM_ENAN on a non-finite
 * velocity (the state is then unchanged). */
int nm_explicit_step(nm_ctx* ctx, const double* Udot, int per_point, int n_steps, nm_step_stats* st);

/* Largest eigenvalue omega^2 of the discrete problem K x = omega^2 rho x with
 * K = -div(C : grad^s .) (section 2.3.3: "solving the discrete eigenvalue problem" for
 * a heterogeneous medium), by power iteration on rho^-1 K.  x_dev: device FP64 3 x N start
 * vector, overwritten by the last iterate (unit rho-weighted norm).  *omega2 receives the
 * Rayleigh quotient x.Kx / x.rho x after `iters` products (a lower bound of omega_max^2 that
 * approaches it as iters grows).  Any context; synchronous. */
int nm_omega2_max(nm_ctx* ctx, void* x_dev, int iters, double* omega2);

/* Au = A(u), eq. (Fourier_ND_A) mapped to real space, unscaled, no Gamma
 * projection.  u_dev / Au_dev: caller-owned device buffers of 3 x N values of
 * the given dtype (NM_FP64 or NM_FP32), SoA, distinct.  Asynchronous on the
 * context stream. */
int nm_apply_operator(nm_ctx* ctx, const void* u_dev, void* Au_dev, int dtype);

/* z = M r with the reference-medium preconditioner of eqs. (precond)-(acous)
 * (no Gamma projection).  Same buffer conventions as nm_apply_operator. */
int nm_precond_apply(nm_ctx* ctx, const void* r_dev, void* z_dev, int dtype);

/* FP64 PCG solve of A x = b on device buffers (3 x N doubles each).  x holds
 * the initial guess and receives the solution.  masked != 0 runs on the free
 * dofs only (Gamma entries of x kept, Gamma rows of b ignored), with the
 * reference norm ||P(b - A xbar)||, xbar = x on Gamma and 0 elsewhere.
 * Stops at ||r|| <= tol * ||b_ref||; fixed_iters >= 0 runs exactly that many
 * iterations instead.  Synchronous.  iters / relres may be NULL. */
int nm_pcg_solve(nm_ctx* ctx, const void* b_dev, void* x_dev, int masked, double tol, int max_iter, int fixed_iters,
                 int* iters, double* relres);

/* Checkpoint: host copies of u, v, a (dim x N each, any may be NULL), the last
 * Gamma force F (dim*n_gamma, may be NULL) and the step count. */
int nm_get_state(const nm_ctx* ctx, double* u, double* v, double* a, double* F_gamma, int64_t* step);
/* Restore a checkpoint taken by nm_get_state (u, v, a required). */
int nm_set_state(nm_ctx* ctx, const double* u, const double* v, const double* a, int64_t step);
/* Zero-copy device views of the state (3 x N doubles each), valid until the next
 * step (steps swap the displacement buffers); writes through them are seen by the
 * next step. */
int nm_state_device_ptrs(nm_ctx* ctx, void** u, void** v, void** a);
/* The Green matrix (d*n_gamma)^2, row major, before factorization; GREEN route only.
 * Stored and passed back through nm_options.green_in it replaces the unit-force solves. */
int nm_green_matrix(const nm_ctx* ctx, double* G);
/* X = G^-1 V (host vectors of d*n_gamma values) with the LU factors the context holds on
 * the device (the solve of eq. L-determination_ND without the 1/(beta dt^2)); GREEN
 * route only.  Synchronous. */
int nm_green_solve(nm_ctx* ctx, const double* V, double* X);

/* Measurement: run the passes of one operator apply (which == 0: seven passes)
 * or one preconditioner apply (which == 1: five passes) reps times on the
 * context stream, with a HIP event pair around every pass; ms[i] receives the
 * average duration of pass i in chain order (ms needs 9 entries).  Buffers as
 * for nm_apply_operator.  Synchronous. */
int nm_profile_passes(nm_ctx* ctx, int which, const void* u_dev, void* out_dev, int dtype, int reps, double* ms);

/* ------------------------------------------------------------------------
 * Learned warm start (an addition to the paper's method): a periodic 3D
 * convolutional network, 4 layers of 3x3x3 kernels, 16 hidden channels,
 * leaky ReLU (slope 0.1), BF16 weights and activations with FP32
 * accumulation on the matrix cores.  It predicts the correction to the
 * Newmark predictor u~ = u_n + dt v_n + dt^2 (1/2 - beta) a_n:
 *     x0 = u~ + s * net(f),   s = rms(u~ - u_n),
 * with per-voxel features f (BF16, 32 channels, channels-last [N][32]):
 * u_n/s, dt v_n/s, dt^2 (1/2 - beta) a_n/s (the Newmark state),
 * rho/rhobar, C_voigt/Cbar_11 (21), 0.
 * The Krylov solve still runs to the same tolerance; only the initial
 * iterate changes.  Grids for the network: every axis a power of two and
 * n1 >= 16.  A network object is independent of any solver context.
 * ------------------------------------------------------------------------ */
typedef struct nm_net nm_net;

/* Create a network with seeded random weights (FP32 master copy on the device). */
int nm_net_create(unsigned long long seed, nm_net** out);
void nm_net_destroy(nm_net* net);
/* Number of FP32 parameters: per layer W[cout][cin][3][3][3] (taps z, y, x) then b[cout];
 * layers 31->16->16->16->3. */
long nm_net_num_params(const nm_net* net);
int nm_net_get_params(const nm_net* net, float* w);
/* Replace the parameters (host FP32); resets the optimizer state. */
int nm_net_set_params(nm_net* net, const float* w);
/* pred (device FP32 [N][4], components 0..2) = net(feat) for features feat (device BF16 [N][32]). */
int nm_net_forward(nm_net* net, void* hip_stream, const int* grid, const void* feat_dev, void* pred_dev);
/* One Adam step (lr, beta1 0.9, beta2 0.999) on the mean squared error between
 * net(feat) and target (device FP32 [N][4]); loss (may be NULL) receives the
 * loss before the update.  Synchronous. */
int nm_net_train_step(nm_net* net, void* hip_stream, const int* grid, const void* feat_dev, const void* target_dev,
                      float lr, float* loss);
/* Gradients of that loss with respect to every parameter (host FP32, nm_net_num_params entries). */
int nm_net_gradients(nm_net* net, void* hip_stream, const int* grid, const void* feat_dev, const void* target_dev,
                     float* grad_host, float* loss);
/* One periodic 3x3x3 convolution layer on caller buffers (checks of the matrix-core kernels).
 * Weights w: host FP32 [cout][cin][27]; bias host FP32 [cout] or NULL.
 *   mode 0: out (device FP32 [N][16]) = conv(x), x device BF16 [N][cinp]
 *   mode 1: out (device FP32 [N][16]) = transposed conv of dy (device BF16 [N][16]); cinp == 16
 *   mode 2: dw_host [cout][cin][27], db_host [cout] = weight and bias gradients for input x and dy
 * cinp is 16 or 32, cin <= cinp, cout <= 16.  Synchronous. */
int nm_conv3d_bf16(void* hip_stream, int mode, const int* grid, int cinp, int cin, int cout, const void* x_dev,
                   const void* w_fp32_host, const float* bias_host, const void* dy_dev, void* out_dev, float* dw_host,
                   float* db_host);

/* nm_conv3d_bf16 for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same arguments,
 * kernels and results, with every device buffer of the call (FP32 and packed BF16 weights,
 * bias, weight-gradient partial sums) taken from one file-scope device array of 16 MiB
 * that each device holds until the process ends.  It calls no hipMalloc or hipFree.  The
 * weight-gradient pass (mode 2) uses at most 256 partial-sum slots, so the array does not
 * grow with the grid and no grid accepted by nm_conv3d_bf16 is too large; its sums are
 * grouped differently from nm_conv3d_bf16's (FP32 rounding differs, modes 0 and 1 are
 * identical).  Every call on a device shares that device's array and leaves its contents
 * behind: calls that overlap on one device race.  Synchronous on hip_stream. */
int nm_conv3d_bf16_noalloc(void* hip_stream, int mode, const int* grid, int cinp, int cin, int cout,
                           const void* x_dev, const void* w_fp32_host, const float* bias_host, const void* dy_dev,
                           void* out_dev, float* dw_host, float* db_host);

/* Attach a network to a solver context (not owned; NULL detaches).  Needed by
 * NM_WS_LEARNED and by the two training-sample calls below. */
int nm_ws_attach(nm_ctx* ctx, nm_net* net);
/* Between steps: features (device BF16 [N][32]) of the next step from the current
 * Newmark state (u_n, v_n, a_n); stores the scale s in the context. */
int nm_ws_features(nm_ctx* ctx, void* feat_dev);
/* The learned initial iterate x0 = u~ + s net(f) of the coming step (device FP64 SoA
 * 3 x N; Gamma entries not yet replaced by U), as NM_WS_LEARNED computes it inside
 * nm_newmark_step (the material share of the first layer cached per network version). */
int nm_ws_predict(nm_ctx* ctx, void* x0_dev);
/* After the following nm_newmark_step: the training target (u_{n+1} - u~) / s as
 * device FP32 [N][4]. */
int nm_ws_target(nm_ctx* ctx, void* target_dev);

/* Residual-norm training of the learned start.  The Krylov solve measures the
 * projected residual, so the network can be trained on it directly: with
 * x0 = u~_Gamma + s P net(f) (u~_Gamma: the predictor with U(t_{n+1}) on Gamma;
 * P zeroes Gamma voxels) and r0 = P (b - A x0) = rp - s P A P net(f),
 *     metric 0:  L = |r0|^2 / cref,            cref  = |r_bar|^2,
 *     metric 1:  L = r0 . (P M P r0) / crefM,   crefM = r_bar . (P M P r_bar),
 * rp = P (b - A u~_Gamma), r_bar = P (b - A u_bar) (the reference residual of the
 * projected solve); A is the operator of eq. (Fourier_ND_A), b that of eq.
 * (Fourier_ND_b), M the preconditioner of eqs. (precond)-(acous).  Metric 1 weighs
 * the error roughly in the energy norm that conjugate gradients reduce.
 * Projected route only.
 *
 * Sample (between steps, before the step to t_{n+1}): features (device BF16
 * [N][32]), rp (device FP64 SoA 3 x N), s, cref and crefM (host; crefM may be
 * NULL).  U_next as for nm_newmark_step.  The solver state is unchanged. */
int nm_ws_residual_sample(nm_ctx* ctx, const double* U_next, int per_point, void* feat_dev, void* rp_dev,
                          double* s_out, double* cref_out, double* crefM_out);
/* One Adam step (lr) of the attached network on L (metric 0 or 1, with the
 * matching reference value) for a sample of this context's problem; loss (may
 * be NULL) receives L before the update.  Synchronous; the solver state is
 * unchanged. */
int nm_ws_train_residual(nm_ctx* ctx, const void* feat_dev, const void* rp_dev, double s, double cref, int metric,
                         float lr, float* loss);

/* The HIP stream (hipStream_t) all of the context's work is queued on. */
void* nm_get_stream(nm_ctx* ctx);

const char* nm_last_error(const nm_ctx* ctx);
void nm_destroy(nm_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* NEWMARK_H */
