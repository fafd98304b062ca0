// C ABI and solver orchestration: Newmark time stepping (eq. Newmark,
// Algorithm 2), preconditioned conjugate gradients on the FFT operator
// (section 2.2.3), the Gamma constraint by the Green-matrix route (eqs.
// (f_discrete)-(L-determination_ND)) or by projection onto the free dofs,
// and FP32/FP64 mixed precision by iterative refinement.
#include "../../include/newmark.h"
#include "nm_common.h"
#include "nm_fft.h"
#include "nm_passes.h"
#include "nm_vec.h"
#include "nm_net.h"
#include "nm_green.h"

#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

using namespace nm;

// Padding (complex elements) of the half-spectrum plane and component strides.
#ifndef NM_PAD_PLANE
#define NM_PAD_PLANE 0
#endif
#ifndef NM_PAD_COMP
#define NM_PAD_COMP 1040
#endif

struct nm_ctx {
    // problem
    int dim = 3, n1 = 0, n2 = 0, n3 = 0, nph = 0;
    long N = 0, NS = 0, ng = 0;
    SpecLayout lay{};
    double dt = 0, beta = 0.25, gam = 0.5;
    std::vector<int64_t> gidx_h;
    nm_options opt{};
    SpecParams sp{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int route = NM_ROUTE_PROJECTED;
    // device problem data
    uint16_t* phase = nullptr;
    uint8_t* mask = nullptr;
    int64_t* gidx = nullptr;
    double* C64 = nullptr;
    float* C32 = nullptr;
    double* rho64 = nullptr;   // operator density rho + gamma dt c (rho without damping)
    float* rho32 = nullptr;
    double* rhot64 = nullptr;  // true density (aliases rho64 without damping)
    double* damp64 = nullptr;  // viscous coefficient c per phase, or null
    double2* tw64 = nullptr;
    float2* tw32 = nullptr;
    // scalars and reductions
    double* scal = nullptr;
    double* hscal = nullptr; // pinned host mirror
    double* part_a = nullptr;
    double* part_b = nullptr;
    int npart = 0;
    // FP64 fields (3 x N each)
    double *u = nullptr, *v = nullptr, *a = nullptr, *ut = nullptr, *b = nullptr, *w = nullptr;
    double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *uf = nullptr;
    double2* spec64 = nullptr;
    double2* spec64b = nullptr;
    // FP32 fields
    float *d32 = nullptr, *r32 = nullptr, *p32 = nullptr, *q32 = nullptr;
    float2* spec32 = nullptr;
    float2* spec32b = nullptr;
    // Gamma buffers
    double* Ubuf = nullptr; // dim * max(ng, 1)
    double* lift = nullptr; // projected route: A e_c, e_c = unit component c on Gamma (3 x (3 x N))
    bool pred_ready = false; // ut and b hold the predictor of the coming step (and winc its scale sums)
    double* winc = nullptr;  // per-block sums of |u~ - u_n|^2 from the fused corrector
    bool d32_is_x = false;   // d32 holds the FP32 copy of the initial iterate (learned start)
    long ws_rejected = 0;    // steps whose learned iterate was replaced by the zero start
    uint16_t* sfeat = nullptr; // unscaled BF16 state features [N][16] of the learned start
    hipEvent_t ev_warm[2] = {nullptr, nullptr}; // brackets the learned start on the stream (timing only)
    bool sfeat_ready = false;  // sfeat was written by the last fused corrector
    double* gbuf = nullptr; // dim * max(ng, 1)
    std::vector<double> G, F_last; // G: host copy (row major) for nm_green_matrix
    double* Gdev = nullptr;        // G, then its LU factors (column major, d n_gamma square)
    int* pivdev = nullptr;         // row swaps of the factorization
    int* permdev = nullptr;        // the swaps composed into one row permutation
    double* dinvdev = nullptr;     // inverted 256 x 256 diagonal blocks of the factors
    double* luwork = nullptr;      // 2 x (d n_gamma) work vector of the substitutions
    int* singdev = nullptr;        // set by the factorization on a zero pivot
    int green_sweeps = 0, green_inner = 0; // mixed-precision Green route: running totals
    // several unit-force solves at once (Green route preprocessing): fields [b][3][N] and
    // spectra [b][6 cs] of up to mnb solves, their partial sums and scalar blocks
    int mnb = 0;
    double *mX = nullptr, *mR = nullptr, *mP = nullptr, *mQ = nullptr, *mU = nullptr, *mB = nullptr;
    double2 *mS = nullptr, *mS2 = nullptr;
    float *mD32 = nullptr, *mR32 = nullptr, *mP32 = nullptr, *mQ32 = nullptr; // mixed precision
    float2 *mS32 = nullptr, *mS2_32 = nullptr;
    double *mpa = nullptr, *mpb = nullptr, *mscal = nullptr, *mhscal = nullptr;
    // explicit central-difference scheme (beta == 0)
    bool explicit_scheme = false;
    double* Fdev = nullptr;      // dim * max(ng, 1): the Gamma force of the last explicit step
    bool F_on_device = false;    // F_last is stale; Fdev holds the force
    double* ubatch = nullptr;    // prescribed velocities of a batch of explicit steps
    size_t ubatch_cap = 0;
    int64_t step = 0;
    std::string err;
    std::vector<void*> allocs;
    // learned warm start (network attached by nm_ws_attach, not owned)
    nm_net* net = nullptr;
    uint16_t* feat = nullptr;
    float* matf = nullptr;
    double* wscale = nullptr;
    double* wred = nullptr;
    uint16_t* l0mat = nullptr; // BF16 [N][16]
    unsigned long long l0mat_version = 0;
};

namespace {

int fail(nm_ctx* c, int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}

#define HIPCHK(c, expr)                                                                                                \
    do {                                                                                                               \
        hipError_t e_ = (expr);                                                                                        \
        if (e_ != hipSuccess) return fail((c), NM_EHIP, "%s: %s", #expr, hipGetErrorString(e_));                      \
    } while (0)
#define LCHK(c, expr)                                                                                                  \
    do {                                                                                                               \
        int e_ = (expr);                                                                                               \
        if (e_ != 0) {                                                                                                 \
            hipError_t he_ = hipGetLastError();                                                                        \
            return fail((c), e_ == -1 ? NM_EUNSUPPORTED : NM_EHIP, "%s failed (%s)", #expr, hipGetErrorString(he_));   \
        }                                                                                                              \
    } while (0)
#define CHK(expr)                                                                                                      \
    do {                                                                                                               \
        int e_ = (expr);                                                                                               \
        if (e_ != NM_OK) return e_;                                                                                    \
    } while (0)

template <typename T> int dalloc(nm_ctx* c, T** ptr, size_t count)
{
    void* p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc(&p, count * sizeof(T));
    if (e != hipSuccess) {
        *ptr = nullptr;
        return fail(c, NM_ENOMEM, "hipMalloc of %zu bytes failed: %s", count * sizeof(T), hipGetErrorString(e));
    }
    c->allocs.push_back(p);
    *ptr = (T*)p;
    return NM_OK;
}

// Release a buffer from dalloc before the context ends.
template <typename T> void dfree(nm_ctx* c, T** ptr)
{
    if (!*ptr) return;
    for (size_t i = 0; i < c->allocs.size(); i++)
        if (c->allocs[i] == (void*)*ptr) {
            (void)hipFree(*ptr);
            c->allocs.erase(c->allocs.begin() + i);
            break;
        }
    *ptr = nullptr;
}

bool pow2_in(int n, int lo, int hi) { return n >= lo && n <= hi && (n & (n - 1)) == 0; }

template <typename T> struct Prec;
template <> struct Prec<double> {
    static const void* tw(nm_ctx* c) { return c->tw64; }
    static const void* C(nm_ctx* c) { return c->C64; }
    static const void* rho(nm_ctx* c) { return c->rho64; }
    static void* spec(nm_ctx* c) { return c->spec64; }
    static void* spec2(nm_ctx* c) { return c->spec64b; }
};
template <> struct Prec<float> {
    static const void* tw(nm_ctx* c) { return c->tw32; }
    static const void* C(nm_ctx* c) { return c->C32; }
    static const void* rho(nm_ctx* c) { return c->rho32; }
    static void* spec(nm_ctx* c) { return c->spec32; }
    static void* spec2(nm_ctx* c) { return c->spec32b; }
};

XFwdArgs xf_args(nm_ctx* c, void* spec)
{
    XFwdArgs a{};
    a.spec = spec;
    a.lay = c->lay;
    a.scal = c->scal;
    a.nlines = 3L * c->n2 * c->n3;
    return a;
}
XInvArgs xi_args(nm_ctx* c, void* spec, void* out, const void* aux, const void* rho, const uint8_t* mask,
                 double* partials)
{
    XInvArgs a{};
    a.spec = spec;
    a.lay = c->lay;
    a.out = out;
    a.aux = aux;
    a.phase = c->phase;
    a.rho = rho;
    a.mask = mask;
    a.partials = partials;
    a.nlines = 3L * c->n2 * c->n3;
    a.lines_per_comp = (long)c->n2 * c->n3;
    a.dim = c->dim;
    return a;
}

// The six passes of q = A p after the x-forward one (which left the x spectrum of p in S).
// xmode: the fused stage of the last pass; bdt2 (when not NaN) replaces beta dt^2 in the
// scale -beta dt^2 of the divergence, so that the chain yields -bdt2 div sigma (+ rho p).
template <typename T>
int chain_operator_rest(nm_ctx* c, const XInvArgs& ia, int xmode = XI_OPERATOR, double bdt2 = NAN)
{
    hipStream_t s = c->stream;
    void* spec = Prec<T>::spec(c);
    void* spec2 = Prec<T>::spec2(c);
    const void* tw = Prec<T>::tw(c);
    const SpecLayout& lay = ia.lay;
    SpecParams sp = c->sp;
    sp.stop = lay.stop;
    if (!std::isnan(bdt2)) sp.bdt2 = bdt2;
    LCHK(c, launch_colop<T>(YOP_DERIV, sp, lay, spec, spec2, tw, s));
    LCHK(c, launch_colop<T>(ZOP_STRAIN, sp, lay, spec, spec2, tw, s));
    LCHK(c, launch_xstress<T>(c->n1, spec2, lay, c->phase, Prec<T>::C(c), tw, s));
    LCHK(c, launch_colop<T>(YOP_DIV, sp, lay, spec, spec2, tw, s));
    LCHK(c, launch_colop<T>(ZOP_DIVZ, sp, lay, spec, spec2, tw, s));
    LCHK(c, launch_xinv<T>(xmode, c->n1, ia, tw, s));
    return NM_OK;
}

// q = A p as seven passes: x-forward (3), D_y (3 -> 3), strain (6), x-inverse +
// sigma = C : eps + x-forward (6), y part of the divergence, z part of the
// divergence, x-inverse + rho p.  S and S2 are the two half-spectrum buffers.
// The layout in fa carries the loop's stop flag (null outside a batched Krylov loop);
// every pass of the chain gets it.
template <typename T> int chain_operator(nm_ctx* c, int fmode, const XFwdArgs& fa, const XInvArgs& ia)
{
    LCHK(c, launch_xfwd<T>(fmode, c->n1, fa, Prec<T>::tw(c), c->stream));
    return chain_operator_rest<T>(c, ia);
}

// z = M r up to the x-inverse: x/y/z forward, pointwise (beta dt^2 K + rhobar I)^-1,
// z and y inverse; the x spectrum of z is left in S.  partials (or null): per-block
// sums of r . z taken on the spectrum inside the z pass.
template <typename T> int chain_precond_spec(nm_ctx* c, int fmode, const XFwdArgs& fa, double* partials)
{
    hipStream_t s = c->stream;
    void* spec = Prec<T>::spec(c);
    const void* tw = Prec<T>::tw(c);
    const SpecLayout& lay = fa.lay;
    SpecParams sp = c->sp;
    sp.stop = lay.stop;
    LCHK(c, launch_xfwd<T>(fmode, c->n1, fa, tw, s));
    LCHK(c, launch_ypass<T>(-1, 3, lay, spec, tw, s));
    LCHK(c, launch_zprecond<T>(sp, lay, spec, tw, s, partials));
    LCHK(c, launch_ypass<T>(+1, 3, lay, spec, tw, s));
    return NM_OK;
}

// z = M r: x/y/z forward, pointwise (beta dt^2 K + rhobar I)^-1, inverse.
template <typename T> int chain_precond(nm_ctx* c, int fmode, const XFwdArgs& fa, const XInvArgs& ia)
{
    // with ia.partials the product r . z is summed on the spectrum inside the z pass, so
    // the final x pass need not read r again
    XInvArgs ib = ia;
    if (ia.partials) {
        ib.partials = nullptr;
        ib.aux = nullptr;
    }
    CHK(chain_precond_spec<T>(c, fmode, fa, ia.partials));
    LCHK(c, launch_xinv<T>(XI_PRECOND, c->n1, ib, Prec<T>::tw(c), c->stream));
    return NM_OK;
}

// q = A x (optionally masked), no reduction.
template <typename T> int apply_A(nm_ctx* c, const T* x, T* out, const uint8_t* mask)
{
    XFwdArgs fa = xf_args(c, Prec<T>::spec(c));
    fa.src = x;
    XInvArgs ia = xi_args(c, Prec<T>::spec(c), out, x, Prec<T>::rho(c), mask, nullptr);
    return chain_operator<T>(c, XF_PLAIN, fa, ia);
}

// out = scale * div(C : grad^s x) (FP64, no inertia term, no Gamma projection).
int div_stress(nm_ctx* c, const double* x, double* out, double scale)
{
    XFwdArgs fa = xf_args(c, c->spec64);
    fa.src = x;
    XInvArgs ia = xi_args(c, c->spec64, out, x, c->rho64, nullptr, nullptr);
    LCHK(c, launch_xfwd<double>(XF_PLAIN, c->n1, fa, c->tw64, c->stream));
    return chain_operator_rest<double>(c, ia, XI_PLAIN, -scale);
}

int read_scalars(nm_ctx* c)
{
    HIPCHK(c, hipMemcpyAsync(c->hscal, c->scal, S_COUNT * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return NM_OK;
}

// ||x||^2 of a 3 x N field (deterministic), returned on the host.
template <typename T> int norm2(nm_ctx* c, const T* x, double* out)
{
    const long n = 3 * c->N;
    LCHK(c, launch_dot<T>(x, x, n, c->part_a, c->stream));
    LCHK(c, launch_reduce(c->part_a, vec_blocks(n), c->scal, RED_STORE_SLOT, 6, c->stream));
    CHK(read_scalars(c));
    *out = c->hscal[6];
    return NM_OK;
}

struct PcgResult {
    int iters = 0;
    double rr = 0;
    double rr0 = 0;
    bool converged = false;
};

// Preconditioned conjugate gradients (Hestenes-Stiefel) on real-space vectors.
// x: initial guess / solution.  With masked, P A P and P M P on the free dofs.
// rr_known >= 0: r already holds P (rhs - A x) with r.r = rr_known (no initial apply;
// rhs may then be null).  The preconditioned residual z lives only as the x spectrum
// between the preconditioner's z pass and the next direction update.
template <typename T>
int pcg(nm_ctx* c, const T* rhs, T* x, T* r, T* p, T* q, bool masked, bool x_zero, double bref, double tol,
        int max_iter, int fixed_iters, bool allow_unconverged, PcgResult* res, double rr_known = -1.0,
        double* x64 = nullptr)
{
    hipStream_t s = c->stream;
    const uint8_t* mk = masked ? c->mask : nullptr;
    const long n = 3 * c->N;
    void* spec = Prec<T>::spec(c);
    // r = P (b - A x)
    double rr = rr_known;
    if (rr_known < 0 && !rhs) return fail(c, NM_EINVAL, "PCG needs the right-hand side or the initial residual");
    if (rr_known < 0) {
        if (x_zero) LCHK(c, launch_fill<T>(q, (T)0, n, s));
        else CHK(apply_A<T>(c, x, q, mk));
        LCHK(c, launch_residual<T>(rhs, q, r, mk, c->N, 3, c->part_a, s));
        LCHK(c, launch_reduce(c->part_a, vec_blocks(n), c->scal, RED_STORE_RR, 0, s));
        CHK(read_scalars(c));
        rr = c->hscal[S_RR];
    }
    res->iters = 0;
    res->rr = rr;
    res->rr0 = rr;
    if (!std::isfinite(rr)) return fail(c, NM_ENAN, "non-finite initial residual");
    if (bref <= 0) bref = 1.0;
    const double thr = tol * bref;
    if ((fixed_iters < 0 && rr <= thr * thr) || fixed_iters == 0) {
        res->converged = true;
        return NM_OK;
    }
    const int nb = xinv_blocks(c->n1, 3L * c->n2 * c->n3);
    const int nbz = zprecond_blocks<T>(c->sp);
    // z = P M r as its x spectrum (the x-inverse is fused into the first p update), rz = r.z
    {
        XFwdArgs fa = xf_args(c, spec);
        fa.src = r;
        CHK(chain_precond_spec<T>(c, XF_PLAIN, fa, c->part_b));
        LCHK(c, launch_reduce(c->part_b, nbz, c->scal, RED_RZ_INIT, 0, s));
    }
    // Iterations run in batches on the device: the residual reduction of each iteration
    // counts it and raises the stop flag when the loop is done, after which every
    // guarded kernel returns at once; the host reads the scalars once per batch and sizes
    // the next batch from the observed convergence rate.
    const double thr2 = thr * thr;
    const bool fixed = fixed_iters >= 0;
    LCHK(c, launch_loop_init(c->scal, thr2, fixed ? fixed_iters : max_iter, fixed ? 1 : 0, s));
    const double* stop = c->scal + S_STOP;
    // first batch: 70% of the iterations a reduction of 4 per iteration would need (the
    // reference-medium preconditioner does better than that on these media), 1 .. 6
    int it = 0, batch = 1;
    if (fixed) {
        batch = fixed_iters;
    } else if (rr > thr2 && thr2 > 0) {
        const double need = 0.5 * std::log(rr / thr2) / std::log(4.0);
        batch = (int)std::floor(0.7 * need);
        batch = batch < 1 ? 1 : (batch > 6 ? 6 : batch);
    }
    double rr_prev = rr;
    int it_prev = 0;
    for (;;) {
        for (int k = 0; k < batch; k++) {
            // z = P x-inv(Z); p = z + beta p (x += alpha p_old) with its x spectrum;
            // q = P A p ; alpha = rz / p.q
            {
                XInvArgs pa = xi_args(c, spec, nullptr, nullptr, nullptr, mk, nullptr);
                pa.lay.stop = stop;
                pa.p = p;
                pa.x = x;
                pa.scal = c->scal;
                LCHK(c, launch_xpupdate<T>(c->n1, pa, Prec<T>::tw(c), s));
                XInvArgs ia = xi_args(c, spec, q, p, Prec<T>::rho(c), mk, c->part_b);
                ia.lay.stop = stop;
                CHK(chain_operator_rest<T>(c, ia));
                LCHK(c, launch_reduce(c->part_b, nb, c->scal, RED_ALPHA, 0, s, true));
            }
            // r -= alpha q ; r.r (iteration count, stop test) ; Z = M r with r.z on the
            // spectrum ; beta = r.z_new / r.z_old   (x += alpha p follows in the next p update)
            {
                XFwdArgs fa = xf_args(c, spec);
                fa.lay.stop = stop;
                fa.r = r;
                fa.q = q;
                fa.partials = c->part_a;
                LCHK(c, launch_xfwd<T>(XF_UPDATE, c->n1, fa, Prec<T>::tw(c), s));
                LCHK(c, launch_reduce(c->part_a, xfwd_blocks(c->n1, 3L * c->n2 * c->n3), c->scal, RED_RR_CHECK, 0,
                                      s, true));
                SpecParams sp = c->sp;
                sp.stop = stop;
                LCHK(c, launch_ypass<T>(-1, 3, fa.lay, spec, Prec<T>::tw(c), s));
                LCHK(c, launch_zprecond<T>(sp, fa.lay, spec, Prec<T>::tw(c), s, c->part_b));
                LCHK(c, launch_ypass<T>(+1, 3, fa.lay, spec, Prec<T>::tw(c), s));
                LCHK(c, launch_reduce(c->part_b, nbz, c->scal, RED_BETA, 0, s, true));
            }
        }
        CHK(read_scalars(c));
        it = (int)c->hscal[S_ITER];
        rr = c->hscal[S_RR];
        res->iters = it;
        res->rr = rr;
        if (!std::isfinite(rr)) return fail(c, NM_ENAN, "non-finite residual at iteration %d", it);
        if (c->hscal[S_STOP] != 0.0) {
            // the last iteration's x += alpha p (FP32 with x64: folded into x64 += x + alpha p,
            // x itself left without it)
            if constexpr (std::is_same<T, float>::value) {
                if (x64) LCHK(c, launch_add_f2d_axpy(x64, x, p, c->scal + S_ALPHA, n, s));
                else LCHK(c, launch_axpy_scal<T>(x, p, c->scal + S_ALPHA, n, s));
            } else {
                LCHK(c, launch_axpy_scal<T>(x, p, c->scal + S_ALPHA, n, s));
            }
            if (fixed || rr <= thr2) break;
            if (allow_unconverged) return NM_OK;
            return fail(c, NM_ENOTCONV, "PCG did not reach tol %.3g in %d iterations (rel %.3g)", tol, max_iter,
                        std::sqrt(rr) / bref);
        }
        // next batch: the iterations the observed rate still needs (1 .. 6)
        if (fixed) {
            batch = fixed_iters - it;
        } else {
            double need = 1.0;
            if (it > it_prev && rr > 0 && rr_prev > 0 && rr < rr_prev) {
                const double rate = 0.5 * std::log(rr / rr_prev) / (it - it_prev); // log |r| per iteration
                need = 0.5 * std::log(thr2 / rr) / rate;
            }
            batch = need < 1.0 ? 1 : (need > 6.0 ? 6 : (int)std::floor(need));
        }
        if (batch < 1) batch = 1;
        rr_prev = rr;
        it_prev = it;
    }
    res->converged = true;
    return NM_OK;
}

// ||P (b - A xbar)||, xbar = x on Gamma and 0 elsewhere (reference norm of the projected system).
int projected_bref(nm_ctx* c, const double* x, double* bref)
{
    hipStream_t s = c->stream;
    const long n = 3 * c->N;
    LCHK(c, launch_fill<double>(c->z, 0.0, n, s));
    if (c->ng > 0) {
        LCHK(c, launch_gather_gamma(c->gbuf, x, c->gidx, c->ng, 3, c->N, s));
        LCHK(c, launch_set_gamma(c->z, c->gidx, c->ng, c->gbuf, 1, 3, c->N, s));
    }
    CHK(apply_A<double>(c, c->z, c->q, c->mask));
    LCHK(c, launch_residual<double>(c->b, c->q, c->r, c->mask, c->N, 3, c->part_a, s, c->r32));
    LCHK(c, launch_reduce(c->part_a, vec_blocks(n), c->scal, RED_STORE_RR, 0, s));
    CHK(read_scalars(c));
    *bref = std::sqrt(c->hscal[S_RR]);
    return NM_OK;
}

// The same for a uniform prescribed displacement U3 from the precomputed lifting
// responses (no operator apply); r_bar = P (b - A u_bar) is left in c->r.
int lift_bref(nm_ctx* c, const double* U3, double* bref)
{
    hipStream_t s = c->stream;
    LCHK(c, launch_lift_residual(c->b, c->lift, U3, c->mask, c->N, c->r, c->part_a, s, c->r32));
    LCHK(c, launch_reduce(c->part_a, vec_blocks(3 * c->N), c->scal, RED_STORE_RR, 0, s));
    CHK(read_scalars(c));
    *bref = std::sqrt(c->hscal[S_RR]);
    return NM_OK;
}

// Mixed precision: FP64 residual r = P(b - A x), FP32 PCG correction, x += d.
// Residuals at most this many outer tolerances large are updated with the FP32 operator
// applied to the correction instead of recomputed with the FP64 operator.
constexpr double kSmallUpdate = 5e3;

// rr_known >= 0: c->r already holds the first sweep's residual P (b - A x), r.r = rr_known.
// rejected (or null): set, and nothing solved, when the initial iterate's residual exceeds
// bref (the zero start's), so that the caller can restart from the zero start.
int solve_mixed(nm_ctx* c, double* x, double bref, nm_step_stats* st, double rr_known = -1.0,
                bool* rejected = nullptr)
{
    hipStream_t s = c->stream;
    const long n = 3 * c->N;
    if (bref <= 0) bref = 1.0;
    int sweeps = 0, inner = 0;
    double rr = 0;
    bool small_update = false; // the last correction is small enough for an FP32 residual update
    PcgResult pr;              // the last correction solve
    for (;;) {
        bool approx = false;
        if (sweeps == 0 && rr_known >= 0) {
            rr = rr_known;
        } else if (small_update && pr.converged && pr.rr <= 0.25 * c->opt.tol * c->opt.tol * bref * bref) {
            // the correction solve's recursively updated residual r - P A d (FP32 operator,
            // FP32 updates) stands for the new residual: |r| <= kSmallUpdate tol b_ref, so
            // the operator's FP32 rounding and the updates' (together a few 1e-7 of |r| per
            // iteration) stay below 1e-2 tol b_ref, and a recursive residual at most half
            // the tolerance certifies the FP64 iterate, as the recursive residual of the FP64
            // solve does
            rr = pr.rr;
        } else if (small_update) {
            // r <- r - P A d with the FP32 operator: |A d| is about |r|, at most kSmallUpdate
            // tol b_ref, so its FP32 rounding (a few 1e-7 of |A d|) stays below 1e-2 tol b_ref
            // and the stopping test still certifies the FP64 iterate.  d first takes the
            // solve's last alpha p, which went only into x.
            if (pr.iters > 0) LCHK(c, launch_axpy_scal<float>(c->d32, c->p32, c->scal + S_ALPHA, n, s));
            CHK(apply_A<float>(c, c->d32, c->q32, c->mask));
            LCHK(c, launch_update_f32q(c->r, c->q32, c->mask, c->N, c->part_a, s, c->r32));
            LCHK(c, launch_reduce(c->part_a, vec_blocks(n), c->scal, RED_STORE_RR, 0, s));
            CHK(read_scalars(c));
            rr = c->hscal[S_RR];
        } else if (sweeps == 0) {
            // the first residual only seeds the first correction, whose own accuracy is
            // about inner_tol, so the FP32 operator serves; every later residual (and the
            // stopping test) is FP64
            if (!c->d32_is_x) LCHK(c, launch_cast_d2f(c->d32, x, n, s));
            c->d32_is_x = false;
            CHK(apply_A<float>(c, c->d32, c->q32, c->mask));
            LCHK(c, launch_residual_f32q(c->b, c->q32, c->r, c->mask, c->N, c->part_a, s, c->r32));
            LCHK(c, launch_reduce(c->part_a, vec_blocks(n), c->scal, RED_STORE_RR, 0, s));
            CHK(read_scalars(c));
            rr = c->hscal[S_RR];
            approx = true;
            if (rejected && rr > bref * bref) {
                *rejected = true;
                return NM_OK;
            }
        } else {
            CHK(apply_A<double>(c, x, c->q, c->mask));
            LCHK(c, launch_residual<double>(c->b, c->q, c->r, c->mask, c->N, 3, c->part_a, s, c->r32));
            LCHK(c, launch_reduce(c->part_a, vec_blocks(n), c->scal, RED_STORE_RR, 0, s));
            CHK(read_scalars(c));
            rr = c->hscal[S_RR];
        }
        if (sweeps == 0 && st) st->relres0 = std::sqrt(rr) / bref;
        if (!std::isfinite(rr)) return fail(c, NM_ENAN, "non-finite residual in refinement sweep %d", sweeps);
        if (!approx && std::sqrt(rr) <= c->opt.tol * bref) break;
        if (sweeps >= c->opt.max_sweeps)
            return fail(c, NM_ENOTCONV, "mixed precision did not reach tol %.3g in %d sweeps (rel %.3g)", c->opt.tol,
                        sweeps, std::sqrt(rr) / bref);
        small_update = !approx && std::sqrt(rr) <= kSmallUpdate * c->opt.tol * bref;
        // the correction starts at zero, so its residual is r itself (already P-projected):
        // the FP32 solve starts from its rounded copy, which every residual kernel of this
        // path writes beside r, with the FP64 r.r
        LCHK(c, launch_fill<float>(c->d32, 0.0f, n, s));
        pr = PcgResult{};
        // reduce the residual only as far as the outer tolerance still needs (half of the
        // remaining factor), but never ask FP32 for more than inner_tol
        const double need = 0.5 * c->opt.tol * bref / std::sqrt(rr);
        // x += d, the last PCG update folded in (d itself lacks it)
        CHK(pcg<float>(c, nullptr, c->d32, c->r32, c->p32, c->q32, true, true, std::sqrt(rr),
                       need > c->opt.inner_tol ? need : c->opt.inner_tol, c->opt.max_iter, -1, true, &pr, rr, x));
        inner += pr.iters;
        sweeps++;
    }
    if (st) {
        st->sweeps = sweeps;
        st->inner_iters = inner;
        st->relres = std::sqrt(rr) / bref;
    }
    return NM_OK;
}

// Mixed precision without a Gamma projection (the Green route's solves): FP64 residual
// r = rhs - A x, FP32 PCG correction, x += d, until ||r|| <= tol bref.
// rr_out / rr0_out (or null): the last and the first FP64 residual, squared.
// guard_zero: an initial iterate whose residual exceeds ||rhs|| (the zero start's) is replaced
// by the zero start.
int solve_mixed_plain(nm_ctx* c, const double* rhs, double* x, double bref, double tol, bool x_zero, int* sweeps_out,
                      int* inner_out, double* rr_out = nullptr, double* rr0_out = nullptr, bool guard_zero = false)
{
    hipStream_t s = c->stream;
    const long n = 3 * c->N;
    if (bref <= 0) bref = 1.0;
    int sweeps = 0, inner = 0;
    for (;;) {
        // r = rhs - A x (the first residual of a zero start is rhs itself)
        if (sweeps == 0 && x_zero) LCHK(c, launch_fill<double>(c->q, 0.0, n, s));
        else CHK(apply_A<double>(c, x, c->q, nullptr));
        LCHK(c, launch_residual<double>(rhs, c->q, c->r, nullptr, c->N, 3, c->part_a, s, c->r32));
        LCHK(c, launch_reduce(c->part_a, vec_blocks(n), c->scal, RED_STORE_RR, 0, s));
        CHK(read_scalars(c));
        double rr = c->hscal[S_RR];
        if (!std::isfinite(rr)) return fail(c, NM_ENAN, "non-finite residual in refinement sweep %d", sweeps);
        if (sweeps == 0 && guard_zero && !x_zero && rr > bref * bref) {
            // restart from zero: r = rhs
            LCHK(c, launch_fill<double>(x, 0.0, n, s));
            LCHK(c, launch_fill<double>(c->q, 0.0, n, s));
            LCHK(c, launch_residual<double>(rhs, c->q, c->r, nullptr, c->N, 3, c->part_a, s, c->r32));
            LCHK(c, launch_reduce(c->part_a, vec_blocks(n), c->scal, RED_STORE_RR, 0, s));
            CHK(read_scalars(c));
            rr = c->hscal[S_RR];
            c->ws_rejected++;
        }
        if (sweeps == 0 && rr0_out) *rr0_out = rr;
        if (rr_out) *rr_out = rr;
        if (std::sqrt(rr) <= tol * bref) break;
        if (sweeps >= c->opt.max_sweeps)
            return fail(c, NM_ENOTCONV, "mixed precision did not reach tol %.3g in %d sweeps (rel %.3g)", tol, sweeps,
                        std::sqrt(rr) / bref);
        LCHK(c, launch_fill<float>(c->d32, 0.0f, n, s));
        PcgResult pr;
        const double need = 0.5 * tol * bref / std::sqrt(rr);
        CHK(pcg<float>(c, nullptr, c->d32, c->r32, c->p32, c->q32, false, true, std::sqrt(rr),
                       need > c->opt.inner_tol ? need : c->opt.inner_tol, c->opt.max_iter, -1, true, &pr, rr, x));
        inner += pr.iters;
        sweeps++;
    }
    if (sweeps_out) *sweeps_out += sweeps;
    if (inner_out) *inner_out += inner;
    return NM_OK;
}

// One solve of the Green route (A x = rhs to tol relative to bref, no projection) in the
// context's precision; mixed precision adds its sweeps and FP32 iterations to the
// context's running totals.
// guard_zero (with bref = ||rhs||): an initial iterate whose residual exceeds ||rhs|| is
// replaced by the zero start (the learned start's guard on the Green route's u_b solve).
int green_solve(nm_ctx* c, const double* rhs, double* x, double bref, double tol, bool x_zero, PcgResult* res,
                bool guard_zero = false)
{
    if (c->opt.precision == NM_PREC_MIXED) {
        *res = PcgResult{};
        res->converged = true;
        return solve_mixed_plain(c, rhs, x, bref, tol, x_zero, &c->green_sweeps, &c->green_inner, &res->rr, &res->rr0,
                                 guard_zero);
    }
    double rr0 = -1.0;
    if (guard_zero && !x_zero) {
        const long n = 3 * c->N;
        CHK(apply_A<double>(c, x, c->q, nullptr));
        LCHK(c, launch_residual<double>(rhs, c->q, c->r, nullptr, c->N, 3, c->part_a, c->stream));
        LCHK(c, launch_reduce(c->part_a, vec_blocks(n), c->scal, RED_STORE_RR, 0, c->stream));
        CHK(read_scalars(c));
        rr0 = c->hscal[S_RR];
        if (rr0 > bref * bref) {
            LCHK(c, launch_fill<double>(x, 0.0, n, c->stream));
            LCHK(c, launch_copy<double>(c->r, rhs, n, c->stream));
            rr0 = bref * bref;
            c->ws_rejected++;
        }
    }
    return pcg<double>(c, rhs, x, c->r, c->p, c->q, false, x_zero, bref, tol, c->opt.max_iter, -1, false, res, rr0);
}

// Fields solved together by the Green route's unit-force solves: enough to give the kernels
// about 8M voxels of work (small grids are bound by launches, not by memory traffic), at most
// 16; options.green_batch overrides (1: one at a time).  1 when the launch layout does not keep
// every field's partial sums apart.
int green_batch_size(nm_ctx* c)
{
    int nb = c->opt.green_batch;
    if (nb <= 0) {
        nb = 1;
        while (nb < 16 && (long)nb * 2 * c->N <= (8L << 20)) nb *= 2;
    }
    if (nb > 64) nb = 64;
    const long lpf = 3L * c->n2 * c->n3;
    if (nb < 2 || (long)xfwd_blocks(c->n1, nb * lpf) != (long)nb * xfwd_blocks(c->n1, lpf) ||
        (long)xinv_blocks(c->n1, nb * lpf) != (long)nb * xinv_blocks(c->n1, lpf))
        return 1;
    return nb;
}

// Buffers of nb fields side by side in one precision: real fields [b][3][N], spectra
// [b][6 cs], per-field device scalars.
template <typename T> struct MultiBufs {
    T *x, *r, *p, *q;
    cx_t<T>*S, *S2;
};

// Launch layout of nb fields side by side (3-component passes, the 6-component stress pass,
// the column passes).
struct MultiLayout {
    SpecLayout lay3, lay6;
    SpecParams sp;
    long lpf;
};
MultiLayout multi_layout(nm_ctx* c, int nb)
{
    MultiLayout m;
    m.lpf = 3L * c->n2 * c->n3;
    m.lay3 = c->lay;
    m.lay3.stop = nullptr;
    m.lay3.nb = nb;
    m.lay3.bc = 3;
    m.lay3.bs = 6 * c->lay.cs;
    m.lay6 = m.lay3;
    m.lay6.bc = 1;
    m.sp = c->sp;
    m.sp.stop = nullptr;
    m.sp.bs = 6 * c->lay.cs;
    m.sp.bk = nb;
    return m;
}

// The six passes of q = A p after the x-forward one, for nb fields (S holds their x spectra).
// partials (or null): per-block sums of p.q, field after field.
template <typename T>
int multi_operator_rest(nm_ctx* c, const MultiLayout& L, int nb, const MultiBufs<T>& m, const T* p, T* q,
                        double* partials)
{
    hipStream_t s = c->stream;
    const void* tw = Prec<T>::tw(c);
    LCHK(c, launch_colop<T>(YOP_DERIV, L.sp, L.lay3, m.S, m.S2, tw, s));
    LCHK(c, launch_colop<T>(ZOP_STRAIN, L.sp, L.lay3, m.S, m.S2, tw, s));
    LCHK(c, launch_xstress<T>(c->n1, m.S2, L.lay6, c->phase, Prec<T>::C(c), tw, s));
    LCHK(c, launch_colop<T>(YOP_DIV, L.sp, L.lay3, m.S, m.S2, tw, s));
    LCHK(c, launch_colop<T>(ZOP_DIVZ, L.sp, L.lay3, m.S, m.S2, tw, s));
    XInvArgs ia = xi_args(c, m.S, q, p, Prec<T>::rho(c), nullptr, partials);
    ia.lay = L.lay3;
    ia.nlines = nb * L.lpf;
    ia.lines_per_batch = L.lpf;
    LCHK(c, launch_xinv<T>(XI_OPERATOR, c->n1, ia, tw, s));
    return NM_OK;
}

// nb independent unmasked PCG loops in precision T through one chain of kernels, from x_b = 0
// with the residuals already in m.r: loop b stops on r.r <= thr2[b] (or max_iter) and is
// frozen from then on (the multi-loop reductions: alpha = beta = 0), so that its iterate
// receives the deferred last update once and then stays; loops with frozen[b] start stopped.
// On return every x_b still lacks its deferred last alpha p (alpha is zero for the loops
// frozen before the last iteration); c->mhscal holds the final scalars.
template <typename T>
int pcg_multi_core(nm_ctx* c, int nb, const MultiBufs<T>& m, const double* thr2, const bool* frozen, int max_iter,
                   int* iters_max)
{
    hipStream_t s = c->stream;
    const long n = 3 * c->N;
    const MultiLayout L = multi_layout(c, nb);
    const int nbx = xinv_blocks(c->n1, L.lpf), nbf = xfwd_blocks(c->n1, L.lpf), nbz = zprecond_blocks<T>(c->sp);
    const void* tw = Prec<T>::tw(c);
    for (int b = 0; b < nb; b++) {
        LCHK(c, launch_loop_init(c->mscal + b * S_COUNT, thr2[b], max_iter, 0, s));
        if (frozen[b]) LCHK(c, launch_fill<double>(c->mscal + b * S_COUNT + S_STOP, 1.0, 1, s));
    }
    LCHK(c, launch_fill<T>(m.x, (T)0, nb * n, s));
    // z = M r as its x spectrum, r.z
    XFwdArgs fa{};
    fa.spec = m.S;
    fa.lay = L.lay3;
    fa.scal = c->mscal;
    fa.nlines = nb * L.lpf;
    fa.lines_per_batch = L.lpf;
    fa.src = m.r;
    LCHK(c, launch_xfwd<T>(XF_PLAIN, c->n1, fa, tw, s));
    LCHK(c, launch_ypass<T>(-1, 3 * nb, L.lay3, m.S, tw, s));
    LCHK(c, launch_zprecond<T>(L.sp, L.lay3, m.S, tw, s, c->mpb));
    LCHK(c, launch_ypass<T>(+1, 3 * nb, L.lay3, m.S, tw, s));
    LCHK(c, launch_reduce_multi(c->mpb, nbz, nb, c->mscal, RED_RZ_INIT, s));
    XInvArgs pa = xi_args(c, m.S, nullptr, nullptr, nullptr, nullptr, nullptr);
    pa.lay = L.lay3;
    pa.nlines = nb * L.lpf;
    pa.lines_per_batch = L.lpf;
    pa.p = m.p;
    pa.x = m.x;
    pa.scal = c->mscal;
    XFwdArgs fu = fa;
    fu.src = nullptr;
    fu.r = m.r;
    fu.q = m.q;
    fu.partials = c->mpa;
    int it = 0;
    for (;;) {
        for (int k = 0; k < 4; k++) {
            // p = z + beta p (x += alpha p_old); q = A p; alpha
            LCHK(c, launch_xpupdate<T>(c->n1, pa, tw, s));
            CHK(multi_operator_rest<T>(c, L, nb, m, m.p, m.q, c->mpb));
            LCHK(c, launch_reduce_multi(c->mpb, nbx, nb, c->mscal, RED_ALPHA, s));
            // r -= alpha q, r.r (stop test); z = M r, r.z; beta
            LCHK(c, launch_xfwd<T>(XF_UPDATE, c->n1, fu, tw, s));
            LCHK(c, launch_reduce_multi(c->mpa, nbf, nb, c->mscal, RED_RR_CHECK, s));
            LCHK(c, launch_ypass<T>(-1, 3 * nb, L.lay3, m.S, tw, s));
            LCHK(c, launch_zprecond<T>(L.sp, L.lay3, m.S, tw, s, c->mpb));
            LCHK(c, launch_ypass<T>(+1, 3 * nb, L.lay3, m.S, tw, s));
            LCHK(c, launch_reduce_multi(c->mpb, nbz, nb, c->mscal, RED_BETA, s));
        }
        HIPCHK(c, hipMemcpyAsync(c->mhscal, c->mscal, nb * S_COUNT * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        bool all = true;
        it = 0;
        for (int b = 0; b < nb; b++) {
            const double* h = c->mhscal + b * S_COUNT;
            if (!std::isfinite(h[S_RR])) return fail(c, NM_ENAN, "non-finite residual in unit-force solve %d", b);
            all = all && h[S_STOP] != 0.0;
            it = std::max(it, (int)h[S_ITER]);
        }
        if (all) break;
    }
    if (iters_max) *iters_max = std::max(*iters_max, it);
    return NM_OK;
}

// nb independent unmasked solves A x_b = rhs_b from x_b = 0 (the Green route's unit-force
// solves), c->mB holding the right-hand sides, c->mX receiving the solutions, each to
// ||rhs_b - A x_b|| <= tol ||rhs_b||:
//   FP64: one PCG loop per field; every solution is the one a single FP64 solve gives;
//   mixed: FP64 iterative refinement of FP32 PCG corrections as in the single mixed solve
//   (residual in FP64, correction to max(inner_tol, half the remaining factor), x += d),
//   fields whose FP64 residual has converged frozen in the later corrections.
int solve_multi(nm_ctx* c, int nb, double tol, int* iters_max)
{
    hipStream_t s = c->stream;
    const long n = 3 * c->N;
    std::vector<double> rr(nb), bref(nb), thr2(nb);
    std::vector<char> fz(nb, 0);
    MultiBufs<double> m64{c->mX, c->mR, c->mP, c->mQ, (cx_t<double>*)c->mS, (cx_t<double>*)c->mS2};
    auto residuals = [&](bool x_zero) -> int {
        // R = rhs - A X (FP64; the zero start's residual is rhs itself), its FP32 copy, r.r
        if (!x_zero) {
            const MultiLayout L = multi_layout(c, nb);
            XFwdArgs fa{};
            fa.spec = m64.S;
            fa.lay = L.lay3;
            fa.scal = c->mscal;
            fa.nlines = nb * L.lpf;
            fa.lines_per_batch = L.lpf;
            fa.src = c->mX;
            LCHK(c, launch_xfwd<double>(XF_PLAIN, c->n1, fa, c->tw64, s));
            CHK(multi_operator_rest<double>(c, L, nb, m64, c->mX, c->mQ, nullptr));
        } else {
            LCHK(c, launch_fill<double>(c->mQ, 0.0, nb * n, s));
        }
        for (int b = 0; b < nb; b++) {
            LCHK(c, launch_residual<double>(c->mB + b * n, c->mQ + b * n, c->mR + b * n, nullptr, c->N, 3, c->part_a,
                                            s, c->mR32 ? c->mR32 + b * n : nullptr));
            LCHK(c, launch_reduce(c->part_a, vec_blocks(n), c->mscal + b * S_COUNT, RED_STORE_RR, 0, s));
        }
        HIPCHK(c, hipMemcpyAsync(c->mhscal, c->mscal, nb * S_COUNT * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        for (int b = 0; b < nb; b++) {
            rr[b] = c->mhscal[b * S_COUNT + S_RR];
            if (!std::isfinite(rr[b])) return fail(c, NM_ENAN, "non-finite residual in unit-force solve %d", b);
        }
        return NM_OK;
    };
    CHK(residuals(true));
    for (int b = 0; b < nb; b++) {
        if (!(rr[b] > 0)) return fail(c, NM_EINVAL, "unit-force right-hand side %d is zero", b);
        bref[b] = std::sqrt(rr[b]);
    }
    if (c->opt.precision != NM_PREC_MIXED) {
        for (int b = 0; b < nb; b++) thr2[b] = tol * tol * rr[b];
        const bool none[64] = {};
        CHK(pcg_multi_core<double>(c, nb, m64, thr2.data(), none, c->opt.max_iter, iters_max));
        // the deferred last x += alpha p (zero for the loops frozen before the last iteration)
        for (int b = 0; b < nb; b++) {
            if (!(c->mhscal[b * S_COUNT + S_RR] <= thr2[b]))
                return fail(c, NM_ENOTCONV, "unit-force solve did not reach tol %.3g in %d iterations", tol,
                            (int)c->mhscal[b * S_COUNT + S_ITER]);
            LCHK(c, launch_axpy_scal<double>(c->mX + b * n, c->mP + b * n, c->mscal + b * S_COUNT + S_ALPHA, n, s));
        }
        return NM_OK;
    }
    MultiBufs<float> m32{c->mD32, c->mR32, c->mP32, c->mQ32, (cx_t<float>*)c->mS32, (cx_t<float>*)c->mS2_32};
    LCHK(c, launch_fill<double>(c->mX, 0.0, nb * n, s));
    for (int sweep = 0;; sweep++) {
        if (sweep > 0) CHK(residuals(false));
        bool all = true;
        bool frozen[64];
        for (int b = 0; b < nb; b++) {
            frozen[b] = std::sqrt(rr[b]) <= tol * bref[b];
            all = all && frozen[b];
            const double need = 0.5 * tol * bref[b] / std::sqrt(rr[b]);
            const double t = need > c->opt.inner_tol ? need : c->opt.inner_tol;
            thr2[b] = t * t * rr[b];
        }
        if (all) break;
        if (sweep >= c->opt.max_sweeps)
            return fail(c, NM_ENOTCONV, "mixed precision did not reach tol %.3g in %d sweeps", tol, sweep);
        CHK(pcg_multi_core<float>(c, nb, m32, thr2.data(), frozen, c->opt.max_iter, iters_max));
        // X += D + alpha P (the correction's deferred last update folded in FP64)
        for (int b = 0; b < nb; b++)
            LCHK(c, launch_add_f2d_axpy(c->mX + b * n, c->mD32 + b * n, c->mP32 + b * n,
                                        c->mscal + b * S_COUNT + S_ALPHA, n, s));
    }
    return NM_OK;
}

// G from the unit-force solves of eq. (solve_green): column d p + j is the Gamma trace of
// A^-1 (e_j at x_p), rows ordered d q + i; written into the device matrix column by column
// (no host round trip per column).  With a stored G (row major, as nm_green_matrix returns
// it) the solves are skipped.  Then its LU factors on the device.
int build_green(nm_ctx* c, const double* G_in)
{
    hipStream_t s = c->stream;
    const int d = c->dim;
    const long n = 3 * c->N;
    const long nd = (long)d * c->ng;
    CHK(dalloc(c, &c->Gdev, (size_t)nd * nd));
    CHK(dalloc(c, &c->pivdev, nd));
    CHK(dalloc(c, &c->permdev, nd));
    CHK(dalloc(c, &c->dinvdev, (size_t)((nd + 255) / 256) * 2 * 256 * 256));
    CHK(dalloc(c, &c->luwork, 2 * (size_t)nd));
    CHK(dalloc(c, &c->singdev, 1));
    c->G.assign((size_t)nd * nd, 0.0);
    if (G_in) {
        std::vector<double> cm((size_t)nd * nd); // column major on the device
        for (long i = 0; i < nd; i++)
            for (long j = 0; j < nd; j++) {
                const double v = G_in[(size_t)i * nd + j];
                if (!std::isfinite(v)) return fail(c, NM_EINVAL, "non-finite entry in the stored Green matrix");
                cm[(size_t)j * nd + i] = v;
            }
        std::memcpy(c->G.data(), G_in, c->G.size() * sizeof(double));
        HIPCHK(c, hipMemcpy(c->Gdev, cm.data(), cm.size() * sizeof(double), hipMemcpyHostToDevice));
    } else if (int nb = green_batch_size(c); nb >= 2) {
        // nb unit-force solves at a time in the context's precision
        const bool mixed = c->opt.precision == NM_PREC_MIXED;
        if (c->mnb < nb) {
            const long cs = c->lay.cs;
            const long lpf = 3L * c->n2 * c->n3;
            const int npa = xfwd_blocks(c->n1, lpf);
            const int npb = std::max({xinv_blocks(c->n1, lpf), zprecond_blocks<double>(c->sp),
                                      zprecond_blocks<float>(c->sp)});
            for (double** f : {&c->mX, &c->mR, &c->mP, &c->mQ, &c->mB}) CHK(dalloc(c, f, nb * n));
            CHK(dalloc(c, &c->mU, 3 * (size_t)nb));
            CHK(dalloc(c, &c->mS, nb * 6 * cs));
            CHK(dalloc(c, &c->mS2, nb * 6 * cs));
            if (mixed) {
                for (float** f : {&c->mD32, &c->mR32, &c->mP32, &c->mQ32}) CHK(dalloc(c, f, nb * n));
                CHK(dalloc(c, &c->mS32, nb * 6 * cs));
                CHK(dalloc(c, &c->mS2_32, nb * 6 * cs));
            }
            CHK(dalloc(c, &c->mpa, (size_t)nb * npa));
            CHK(dalloc(c, &c->mpb, (size_t)nb * npb));
            CHK(dalloc(c, &c->mscal, (size_t)nb * S_COUNT));
            HIPCHK(c, hipHostMalloc((void**)&c->mhscal, nb * S_COUNT * sizeof(double), hipHostMallocDefault));
            c->mnb = nb;
        }
        std::vector<double> units(3 * (size_t)nb);
        for (long col0 = 0; col0 < nd; col0 += nb) {
            const int kk = (int)std::min<long>(nb, nd - col0);
            LCHK(c, launch_fill<double>(c->mB, 0.0, kk * n, s));
            std::fill(units.begin(), units.end(), 0.0);
            for (int b = 0; b < kk; b++) units[3 * b + (col0 + b) % d] = 1.0;
            HIPCHK(c, hipMemcpyAsync(c->mU, units.data(), 3 * kk * sizeof(double), hipMemcpyHostToDevice, s));
            for (int b = 0; b < kk; b++)
                LCHK(c, launch_set_gamma(c->mB + b * n, c->gidx + (col0 + b) / d, 1, c->mU + 3 * b, 0, 3, c->N, s));
            int its = 0;
            CHK(solve_multi(c, kk, c->opt.green_tol, &its));
            for (int b = 0; b < kk; b++) {
                LCHK(c, launch_gather_gamma(c->gbuf, c->mX + b * n, c->gidx, c->ng, 3, c->N, s));
                LCHK(c, launch_green_column(c->Gdev, nd, col0 + b, c->gbuf, c->ng, d, s));
            }
            HIPCHK(c, hipStreamSynchronize(s));
            if (c->opt.green_progress) c->opt.green_progress(col0 + kk, nd, c->opt.green_progress_user);
        }
        // the solve buffers are needed only here
        for (double** f : {&c->mX, &c->mR, &c->mP, &c->mQ, &c->mB, &c->mU, &c->mpa, &c->mpb, &c->mscal}) dfree(c, f);
        for (float** f : {&c->mD32, &c->mR32, &c->mP32, &c->mQ32}) dfree(c, f);
        dfree(c, &c->mS);
        dfree(c, &c->mS2);
        dfree(c, &c->mS32);
        dfree(c, &c->mS2_32);
        (void)hipHostFree(c->mhscal);
        c->mhscal = nullptr;
        c->mnb = 0;
        std::vector<double> cm((size_t)nd * nd);
        HIPCHK(c, hipMemcpy(cm.data(), c->Gdev, cm.size() * sizeof(double), hipMemcpyDeviceToHost));
        for (long i = 0; i < nd; i++)
            for (long j = 0; j < nd; j++) c->G[(size_t)i * nd + j] = cm[(size_t)j * nd + i];
    } else {
        double unit[3];
        for (long pnt = 0; pnt < c->ng; pnt++)
            for (int j = 0; j < d; j++) {
                LCHK(c, launch_fill<double>(c->b, 0.0, n, s));
                unit[0] = unit[1] = unit[2] = 0.0;
                unit[j] = 1.0;
                HIPCHK(c, hipMemcpyAsync(c->Ubuf, unit, 3 * sizeof(double), hipMemcpyHostToDevice, s));
                LCHK(c, launch_set_gamma(c->b, c->gidx + pnt, 1, c->Ubuf, 0, 3, c->N, s));
                LCHK(c, launch_fill<double>(c->w, 0.0, n, s));
                PcgResult pr;
                CHK(green_solve(c, c->b, c->w, 1.0, c->opt.green_tol, true, &pr));
                LCHK(c, launch_gather_gamma(c->gbuf, c->w, c->gidx, c->ng, 3, c->N, s));
                LCHK(c, launch_green_column(c->Gdev, nd, d * pnt + j, c->gbuf, c->ng, d, s));
                // unit is a stack buffer that the next copy overwrites
                HIPCHK(c, hipStreamSynchronize(s));
                if (c->opt.green_progress) c->opt.green_progress(d * pnt + j + 1, nd, c->opt.green_progress_user);
            }
        std::vector<double> cm((size_t)nd * nd);
        HIPCHK(c, hipMemcpy(cm.data(), c->Gdev, cm.size() * sizeof(double), hipMemcpyDeviceToHost));
        for (long i = 0; i < nd; i++)
            for (long j = 0; j < nd; j++) c->G[(size_t)i * nd + j] = cm[(size_t)j * nd + i];
    }
    LCHK(c, launch_fill<int>(c->singdev, 0, 1, s));
    LCHK(c, lu_factor_device(c->Gdev, (int)nd, c->pivdev, c->singdev, s));
    int sing = 0;
    HIPCHK(c, hipMemcpyAsync(&sing, c->singdev, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    if (sing) return fail(c, NM_ESINGULAR, "zero pivot in the Green matrix");
    LCHK(c, lu_prepare_solve(c->Gdev, (int)nd, c->pivdev, c->permdev, c->dinvdev, s));
    HIPCHK(c, hipStreamSynchronize(s));
    return NM_OK;
}

void fill_twiddles(std::vector<double2>& t64)
{
    t64.assign(kTwiddleCount, double2{0, 0});
    for (int L = 2; L <= 1024; L *= 2)
        for (int i = 0; i < L; i++) {
            const double ang = -2.0 * M_PI * (double)i / (double)L;
            t64[tw_offset(L) + i] = double2{std::cos(ang), std::sin(ang)};
        }
}

template <typename T> int precond_impl(nm_ctx* c, const T* r, T* z)
{
    XFwdArgs fa = xf_args(c, Prec<T>::spec(c));
    fa.src = r;
    XInvArgs ia = xi_args(c, Prec<T>::spec(c), z, r, Prec<T>::rho(c), nullptr, nullptr);
    return chain_precond<T>(c, XF_PLAIN, fa, ia);
}

// z = P M r (Gamma voxels of the output zeroed), FP64.
int precond_masked(nm_ctx* c, const double* r, double* z)
{
    XFwdArgs fa = xf_args(c, Prec<double>::spec(c));
    fa.src = r;
    XInvArgs ia = xi_args(c, Prec<double>::spec(c), z, r, Prec<double>::rho(c), c->mask, nullptr);
    return chain_precond<double>(c, XF_PLAIN, fa, ia);
}

// x . y of two 3 x N FP64 fields (deterministic), on the host.
int dot64(nm_ctx* c, const double* x, const double* y, double* out)
{
    const long n = 3 * c->N;
    LCHK(c, launch_dot<double>(x, y, n, c->part_a, c->stream));
    LCHK(c, launch_reduce(c->part_a, vec_blocks(n), c->scal, RED_STORE_SLOT, 6, c->stream));
    CHK(read_scalars(c));
    *out = c->hscal[6];
    return NM_OK;
}

// Event-timed passes of one operator (which == 0) or preconditioner (which == 1) apply.
template <typename T> int profile_impl(nm_ctx* c, int which, const T* in, T* out, int reps, double* ms)
{
    hipStream_t s = c->stream;
    void* spec = Prec<T>::spec(c);
    const void* tw = Prec<T>::tw(c);
    const int np = which == 0 ? 7 : 5;
    hipEvent_t ev[10];
    for (int i = 0; i <= np; i++) HIPCHK(c, hipEventCreate(&ev[i]));
    std::vector<double> acc(np, 0.0);
    XFwdArgs fa = xf_args(c, spec);
    fa.src = in;
    const uint8_t* nomask = nullptr;
    XInvArgs ia = xi_args(c, spec, out, in, Prec<T>::rho(c), nomask, nullptr);
    int rc = NM_OK;
    for (int rep = 0; rep < reps && rc == NM_OK; rep++) {
        int k = 0;
        auto mark = [&]() { return hipEventRecord(ev[k++], s) == hipSuccess ? 0 : -2; };
        rc = mark();
        if (which == 0) {
            void* spec2 = Prec<T>::spec2(c);
            rc |= launch_xfwd<T>(XF_PLAIN, c->n1, fa, tw, s) | mark();
            rc |= launch_colop<T>(YOP_DERIV, c->sp, c->lay, spec, spec2, tw, s) | mark();
            rc |= launch_colop<T>(ZOP_STRAIN, c->sp, c->lay, spec, spec2, tw, s) | mark();
            rc |= launch_xstress<T>(c->n1, spec2, c->lay, c->phase, Prec<T>::C(c), tw, s) | mark();
            rc |= launch_colop<T>(YOP_DIV, c->sp, c->lay, spec, spec2, tw, s) | mark();
            rc |= launch_colop<T>(ZOP_DIVZ, c->sp, c->lay, spec, spec2, tw, s) | mark();
            rc |= launch_xinv<T>(XI_OPERATOR, c->n1, ia, tw, s) | mark();
        } else {
            rc |= launch_xfwd<T>(XF_PLAIN, c->n1, fa, tw, s) | mark();
            rc |= launch_ypass<T>(-1, 3, c->lay, spec, tw, s) | mark();
            rc |= launch_zprecond<T>(c->sp, c->lay, spec, tw, s) | mark();
            rc |= launch_ypass<T>(+1, 3, c->lay, spec, tw, s) | mark();
            rc |= launch_xinv<T>(XI_PRECOND, c->n1, ia, tw, s) | mark();
        }
        if (rc != 0) break;
        if (hipEventSynchronize(ev[np]) != hipSuccess) {
            rc = -2;
            break;
        }
        for (int i = 0; i < np; i++) {
            float t = 0;
            (void)hipEventElapsedTime(&t, ev[i], ev[i + 1]);
            acc[i] += t;
        }
    }
    for (int i = 0; i <= np; i++) (void)hipEventDestroy(ev[i]);
    if (rc != 0) return fail(c, NM_EHIP, "pass launch failed during profiling");
    for (int i = 0; i < np; i++) ms[i] = acc[i] / reps;
    return NM_OK;
}

nm::WarmArgs warm_args(nm_ctx* c)
{
    nm::WarmArgs a{};
    a.n1 = c->n1;
    a.n2 = c->n2;
    a.n3 = c->n3;
    a.N = c->N;
    a.u = c->u;
    a.v = c->v;
    a.a = c->a;
    a.ut = c->ut;
    a.dt = c->dt;
    a.c2 = c->dt * c->dt * (0.5 - c->beta);
    a.phase = c->phase;
    a.matf = c->matf;
    a.red = c->wred;
    a.scale = c->wscale;
    a.feat = c->feat;
    a.l0mat = c->l0mat;
    a.l0mat_version = &c->l0mat_version;
    a.sfeat = c->sfeat;
    return a;
}

} // namespace

extern "C" {

const char* nm_last_error(const nm_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

void nm_destroy(nm_ctx* c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (hipEvent_t e : c->ev_warm)
        if (e) (void)hipEventDestroy(e);
    for (void* p : c->allocs) (void)hipFree(p);
    if (c->hscal) (void)hipHostFree(c->hscal);
    if (c->mhscal) (void)hipHostFree(c->mhscal);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

// Lifting responses of the projected route: lift_c = A e_c with e_c the unit
// displacement in component c on every Gamma voxel (zero elsewhere), so that
// A u_bar = sum_c U_c lift_c for a displacement U uniform on Gamma.
static int build_lift(nm_ctx* c)
{
    hipStream_t s = c->stream;
    const long n = 3 * c->N;
    CHK(dalloc(c, &c->lift, 3 * n));
    for (int comp = 0; comp < 3; comp++) {
        const double e[3] = {comp == 0 ? 1.0 : 0.0, comp == 1 ? 1.0 : 0.0, comp == 2 ? 1.0 : 0.0};
        HIPCHK(c, hipMemcpyAsync(c->Ubuf, e, sizeof(e), hipMemcpyHostToDevice, s));
        LCHK(c, launch_fill<double>(c->z, 0.0, n, s));
        LCHK(c, launch_set_gamma(c->z, c->gidx, c->ng, c->Ubuf, 0, 3, c->N, s));
        CHK(apply_A<double>(c, c->z, c->lift + comp * n, nullptr));
        HIPCHK(c, hipStreamSynchronize(s)); // e is a stack buffer and Ubuf is reused
    }
    return NM_OK;
}

static int init_impl(nm_ctx* c, const nm_problem* pb, const nm_options* op)
{
    if (!pb || !op) return fail(c, NM_EINVAL, "null problem or options");
    if (pb->dim != 2 && pb->dim != 3) return fail(c, NM_EUNSUPPORTED, "dim must be 2 or 3");
    c->dim = pb->dim;
    c->n1 = pb->n[0];
    c->n2 = pb->n[1];
    c->n3 = pb->n[2];
    if (!pow2_in(c->n1, 8, 512) || !pow2_in(c->n2, 8, 512))
        return fail(c, NM_EUNSUPPORTED, "n1, n2 must be powers of two in [8, 512]");
    if (c->dim == 2 ? c->n3 != 1 : !pow2_in(c->n3, 8, 512))
        return fail(c, NM_EUNSUPPORTED, "n3 must be 1 in 2D and a power of two in [8, 512] in 3D");
    c->N = (long)c->n1 * c->n2 * c->n3;
    c->NS = c->N / 2;
    {
        int l2 = 0;
        while ((1 << l2) < c->n2) l2++;
        c->lay.M = c->n1 / 2;
        c->lay.n2 = c->n2;
        c->lay.n3 = c->n3;
        c->lay.log2n2 = l2;
        // pad the plane and component strides of large spectra (power-of-two strides
        // make the strided z pass collide in the memory system)
        const long plane = (long)c->n2 * c->lay.M;
        c->lay.ps = plane + (c->n3 > 1 && plane >= 4096 ? NM_PAD_PLANE : 0);
        c->lay.cs = (long)c->n3 * c->lay.ps + (c->N >= (1L << 20) ? NM_PAD_COMP : 0);
    }
    if (pb->n_phases < 1 || pb->n_phases > 65536) return fail(c, NM_EINVAL, "n_phases out of range");
    c->nph = pb->n_phases;
    if (!pb->phase_id || !pb->C_voigt || !pb->rho) return fail(c, NM_EINVAL, "null material arrays");
    if (!(pb->dt > 0) || !(pb->beta >= 0) || !std::isfinite(pb->dt) || !std::isfinite(pb->beta))
        return fail(c, NM_EINVAL, "bad dt or beta");
    c->dt = pb->dt;
    c->beta = pb->beta;
    c->gam = pb->gamma_nm;
    // beta = 0 with gamma = 1/2 is the explicit central-difference scheme (section 2.3)
    c->explicit_scheme = pb->beta == 0.0;
    if (c->explicit_scheme && pb->gamma_nm != 0.5)
        return fail(c, NM_EUNSUPPORTED, "beta = 0 selects the central-difference scheme, which needs gamma = 1/2");
    if (pb->n_gamma < 0 || (pb->n_gamma > 0 && !pb->gamma_idx)) return fail(c, NM_EINVAL, "bad Gamma set");
    c->ng = pb->n_gamma;
    c->gidx_h.assign(pb->gamma_idx, pb->gamma_idx + c->ng);
    for (long i = 0; i < c->ng; i++) {
        if (c->gidx_h[i] < 0 || c->gidx_h[i] >= c->N) return fail(c, NM_EINVAL, "Gamma index %ld out of range", i);
        if (i > 0 && c->gidx_h[i] <= c->gidx_h[i - 1])
            return fail(c, NM_EINVAL, "Gamma indices must be sorted and unique");
    }
    c->opt = *op;
    if (c->explicit_scheme) {
        if (c->opt.precision != NM_PREC_FP64) return fail(c, NM_EUNSUPPORTED, "the explicit scheme runs in FP64");
        if (c->opt.route == NM_ROUTE_GREEN)
            return fail(c, NM_EUNSUPPORTED, "the explicit scheme prescribes the Gamma velocity directly (no Green route)");
        c->opt.tol = c->opt.tol > 0 ? c->opt.tol : 1e-8;
        c->opt.max_iter = c->opt.max_iter > 0 ? c->opt.max_iter : 1;
    }
    if (!(c->opt.tol > 0) || c->opt.max_iter <= 0) return fail(c, NM_EINVAL, "tol and max_iter must be positive");
    if (c->opt.precision == NM_PREC_MIXED) {
        if (!(c->opt.inner_tol > 0)) c->opt.inner_tol = 1e-5;
        if (c->opt.max_sweeps <= 0) c->opt.max_sweeps = 20;
    }
    if (!(c->opt.green_tol > 0)) c->opt.green_tol = c->opt.tol * 1e-2;
    c->route = c->opt.route == NM_ROUTE_GREEN ? NM_ROUTE_GREEN : NM_ROUTE_PROJECTED;
    if (c->opt.warm_start < NM_WS_COLD || c->opt.warm_start > NM_WS_LEARNED)
        return fail(c, NM_EINVAL, "unknown warm start");

    // host-side material checks and reference medium (volume averages)
    std::vector<long> count(c->nph, 0);
    for (long v = 0; v < c->N; v++) {
        if (pb->phase_id[v] >= c->nph) return fail(c, NM_EINVAL, "phase id out of range at voxel %ld", v);
        count[pb->phase_id[v]]++;
    }
    c->sp.L1 = pb->L[0];
    c->sp.L2 = pb->L[1];
    c->sp.L3 = c->dim == 2 ? 1.0 : pb->L[2];
    c->sp.k1 = 2.0 * M_PI / c->sp.L1;
    c->sp.k2 = 2.0 * M_PI / c->sp.L2;
    c->sp.k3 = 2.0 * M_PI / c->sp.L3;
    c->sp.n1 = c->n1;
    c->sp.n2 = c->n2;
    c->sp.n3 = c->n3;
    c->sp.dim = c->dim;
    c->sp.inv_ntot = 1.0 / (double)c->N;
    c->sp.inv_n1 = 1.0 / c->n1;
    c->sp.inv_n2 = 1.0 / c->n2;
    c->sp.inv_n3 = 1.0 / c->n3;
    c->sp.bdt2 = c->beta * c->dt * c->dt;
    // viscous damping (section 5's buffer): M a + C v + K u = f under the same Newmark rule
    // gives the operator density rho + gamma dt c; all-zero coefficients are no damping
    bool damped = false;
    if (pb->damping) {
        for (int g = 0; g < c->nph; g++) {
            if (!(pb->damping[g] >= 0) || !std::isfinite(pb->damping[g]))
                return fail(c, NM_EINVAL, "damping of phase %d must be finite and >= 0", g);
            damped = damped || pb->damping[g] > 0;
        }
        if (damped && c->explicit_scheme)
            return fail(c, NM_EUNSUPPORTED, "viscous damping needs the implicit scheme (beta > 0)");
    }
    std::vector<double> rho_op(pb->rho, pb->rho + c->nph);
    if (damped)
        for (int g = 0; g < c->nph; g++) rho_op[g] = pb->rho[g] + c->gam * c->dt * pb->damping[g];
    c->sp.rhobar = 0;
    for (int k = 0; k < 21; k++) c->sp.Cbar[k] = 0;
    for (int g = 0; g < c->nph; g++) {
        if (!(pb->rho[g] > 0)) return fail(c, NM_EINVAL, "density of phase %d must be positive", g);
        const double wgt = (double)count[g] / (double)c->N;
        c->sp.rhobar += wgt * rho_op[g];
        for (int k = 0; k < 21; k++) {
            if (!std::isfinite(pb->C_voigt[21 * g + k])) return fail(c, NM_EINVAL, "non-finite stiffness");
            c->sp.Cbar[k] += wgt * pb->C_voigt[21 * g + k];
        }
    }
    if (!(pb->L[0] > 0) || !(pb->L[1] > 0) || (c->dim == 3 && !(pb->L[2] > 0)))
        return fail(c, NM_EINVAL, "box lengths must be positive");
    if (pb->diff_rule < NM_DIFF_SPECTRAL || pb->diff_rule > NM_DIFF_CENTRED4)
        return fail(c, NM_EINVAL, "unknown differentiation rule %d", pb->diff_rule);

    // stream
    if (c->stream == nullptr) {
        HIPCHK(c, hipStreamCreate(&c->stream));
        c->own_stream = true;
    }
    hipStream_t s = c->stream;
    const long n = 3 * c->N;
    // device problem data
    CHK(dalloc(c, &c->phase, c->N));
    HIPCHK(c, hipMemcpyAsync(c->phase, pb->phase_id, c->N * sizeof(uint16_t), hipMemcpyHostToDevice, s));
    CHK(dalloc(c, &c->mask, c->N));
    {
        std::vector<uint8_t> m(c->N, 0);
        for (long i = 0; i < c->ng; i++) m[c->gidx_h[i]] = 1;
        HIPCHK(c, hipMemcpy(c->mask, m.data(), c->N, hipMemcpyHostToDevice));
    }
    CHK(dalloc(c, &c->gidx, c->ng));
    if (c->ng) HIPCHK(c, hipMemcpy(c->gidx, c->gidx_h.data(), c->ng * sizeof(int64_t), hipMemcpyHostToDevice));
    {
        std::vector<float> c32(21 * (size_t)c->nph), r32(c->nph);
        for (size_t i = 0; i < c32.size(); i++) c32[i] = (float)pb->C_voigt[i];
        for (int g = 0; g < c->nph; g++) r32[g] = (float)rho_op[g];
        CHK(dalloc(c, &c->C64, 21 * (size_t)c->nph));
        CHK(dalloc(c, &c->C32, 21 * (size_t)c->nph));
        CHK(dalloc(c, &c->rho64, c->nph));
        CHK(dalloc(c, &c->rho32, c->nph));
        HIPCHK(c, hipMemcpy(c->C64, pb->C_voigt, 21 * c->nph * sizeof(double), hipMemcpyHostToDevice));
        HIPCHK(c, hipMemcpy(c->C32, c32.data(), c32.size() * sizeof(float), hipMemcpyHostToDevice));
        HIPCHK(c, hipMemcpy(c->rho64, rho_op.data(), c->nph * sizeof(double), hipMemcpyHostToDevice));
        HIPCHK(c, hipMemcpy(c->rho32, r32.data(), r32.size() * sizeof(float), hipMemcpyHostToDevice));
        c->rhot64 = c->rho64;
        if (damped) {
            CHK(dalloc(c, &c->rhot64, c->nph));
            CHK(dalloc(c, &c->damp64, c->nph));
            HIPCHK(c, hipMemcpy(c->rhot64, pb->rho, c->nph * sizeof(double), hipMemcpyHostToDevice));
            HIPCHK(c, hipMemcpy(c->damp64, pb->damping, c->nph * sizeof(double), hipMemcpyHostToDevice));
        }
    }
    {
        std::vector<double2> t64;
        fill_twiddles(t64);
        std::vector<float2> t32(t64.size());
        for (size_t i = 0; i < t64.size(); i++) t32[i] = float2{(float)t64[i].x, (float)t64[i].y};
        CHK(dalloc(c, &c->tw64, t64.size()));
        CHK(dalloc(c, &c->tw32, t32.size()));
        HIPCHK(c, hipMemcpy(c->tw64, t64.data(), t64.size() * sizeof(double2), hipMemcpyHostToDevice));
        HIPCHK(c, hipMemcpy(c->tw32, t32.data(), t32.size() * sizeof(float2), hipMemcpyHostToDevice));
    }
    if (pb->diff_rule != NM_DIFF_SPECTRAL) {
        // the frequency each bin's derivative uses under the finite-difference rule
        const int na[3] = {c->n1, c->n2, c->n3};
        const double La[3] = {c->sp.L1, c->sp.L2, c->sp.L3};
        std::vector<double> mf;
        for (int ax = 0; ax < 3; ax++) {
            const double h = La[ax] / na[ax];
            for (int k = 0; k < na[ax]; k++) {
                const double th = 2.0 * M_PI * freq_index(k, na[ax]) / na[ax]; // xi h
                mf.push_back(pb->diff_rule == NM_DIFF_CENTRED2 ? std::sin(th) / h
                                                               : (8.0 * std::sin(th) - std::sin(2.0 * th)) / (6.0 * h));
            }
        }
        double* mfd = nullptr;
        CHK(dalloc(c, &mfd, mf.size()));
        HIPCHK(c, hipMemcpy(mfd, mf.data(), mf.size() * sizeof(double), hipMemcpyHostToDevice));
        c->sp.mfreq = mfd;
    }
    CHK(dalloc(c, &c->scal, S_COUNT));
    HIPCHK(c, hipMemset(c->scal, 0, S_COUNT * sizeof(double)));
    HIPCHK(c, hipHostMalloc((void**)&c->hscal, S_COUNT * sizeof(double), hipHostMallocDefault));
    c->npart = std::max({xfwd_blocks(c->n1, 3L * c->n2 * c->n3), vec_blocks(n), zprecond_blocks<double>(c->sp),
                         zprecond_blocks<float>(c->sp)});
    CHK(dalloc(c, &c->part_a, c->npart));
    CHK(dalloc(c, &c->winc, vec_blocks(3 * c->N)));
    CHK(dalloc(c, &c->part_b, c->npart));
    // fields (the explicit scheme keeps only the state and one work field)
    double** f64[] = {&c->u, &c->v, &c->a, &c->q, &c->ut, &c->b, &c->w, &c->r, &c->z, &c->p};
    const int nf64 = c->explicit_scheme ? 4 : 10;
    for (int k = 0; k < nf64; k++) {
        CHK(dalloc(c, f64[k], n));
        LCHK(c, launch_fill<double>(*f64[k], 0.0, n, s));
    }
    CHK(dalloc(c, &c->spec64, 6 * c->lay.cs));
    CHK(dalloc(c, &c->spec64b, 6 * c->lay.cs));
    if (c->route == NM_ROUTE_GREEN && !c->explicit_scheme) {
        CHK(dalloc(c, &c->uf, n));
        LCHK(c, launch_fill<double>(c->uf, 0.0, n, s));
    }
    if (!c->explicit_scheme) {
        CHK(dalloc(c, &c->spec32, 6 * c->lay.cs));
        CHK(dalloc(c, &c->spec32b, 6 * c->lay.cs));
    }
    if (c->explicit_scheme || c->route == NM_ROUTE_GREEN) {
        CHK(dalloc(c, &c->Fdev, c->dim * std::max<long>(c->ng, 1)));
        LCHK(c, launch_fill<double>(c->Fdev, 0.0, c->dim * std::max<long>(c->ng, 1), s));
    }
    if (c->opt.precision == NM_PREC_MIXED) {
        float** f32[] = {&c->d32, &c->r32, &c->p32, &c->q32};
        for (float** f : f32) {
            CHK(dalloc(c, f, n));
            LCHK(c, launch_fill<float>(*f, 0.0f, n, s));
        }
    }
    CHK(dalloc(c, &c->Ubuf, 3 * std::max<long>(c->ng, 1)));
    CHK(dalloc(c, &c->gbuf, 3 * std::max<long>(c->ng, 1)));
    c->F_last.assign(c->dim * c->ng, 0.0);
    // initial state (host dim x N -> device 3 x N); the zero fills queued on the stream
    // above must land before these copies, whatever kind of stream the caller passed
    HIPCHK(c, hipStreamSynchronize(s));
    if (pb->u0) HIPCHK(c, hipMemcpy(c->u, pb->u0, c->dim * c->N * sizeof(double), hipMemcpyHostToDevice));
    if (pb->v0) HIPCHK(c, hipMemcpy(c->v, pb->v0, c->dim * c->N * sizeof(double), hipMemcpyHostToDevice));
    if (pb->u0 && c->explicit_scheme) {
        // a0 = div(C : grad^s u0) / rho
        CHK(div_stress(c, c->u, c->q, 1.0));
        LCHK(c, launch_div_rho(c->a, c->q, c->phase, c->rho64, c->N, s));
    } else if (damped && (pb->u0 || pb->v0)) {
        // a0 = (div(C : grad^s u0) - c v0) / rho
        if (pb->u0) CHK(div_stress(c, c->u, c->q, 1.0));
        LCHK(c, launch_accel0_damped(c->a, pb->u0 ? c->q : nullptr, c->v, c->phase, c->rhot64, c->damp64, c->N, 3, s));
    } else if (pb->u0) {
        // a0 = div(C : grad^s u0) / rho
        CHK(apply_A<double>(c, c->u, c->q, nullptr));
        LCHK(c, launch_accel0(c->a, c->u, c->q, c->phase, c->rho64, c->N, 3, c->sp.bdt2, s));
    }
    if (c->route == NM_ROUTE_GREEN && c->ng > 0 && !c->explicit_scheme) CHK(build_green(c, op->green_in));
    if (c->route == NM_ROUTE_PROJECTED && c->ng > 0 && !c->explicit_scheme) CHK(build_lift(c));
    HIPCHK(c, hipStreamSynchronize(s));
    return NM_OK;
}

int nm_newmark_init(const nm_problem* pb, const nm_options* op, void* hip_stream, nm_ctx** out)
{
    if (!out) return NM_EINVAL;
    *out = nullptr;
    nm_ctx* c = new nm_ctx();
    c->stream = (hipStream_t)hip_stream;
    int st = init_impl(c, pb, op);
    *out = c; // returned even on error so that nm_last_error can be read; caller destroys
    return st;
}

// Prescribed displacement of the coming step: validated, expanded to 3 components
// per point (U3) and copied to the device (Ubuf).
static int upload_U(nm_ctx* c, const double* U_n, int per_point, std::vector<double>& U3)
{
    const int d = c->dim;
    const long nU = per_point ? d * c->ng : d;
    if (c->ng > 0 && !U_n) return fail(c, NM_EINVAL, "null prescribed displacement");
    U3.assign(per_point ? 3 * c->ng : 3, 0.0);
    for (long i = 0; c->ng > 0 && i < nU; i++) {
        if (!std::isfinite(U_n[i])) return fail(c, NM_ENAN, "non-finite prescribed displacement");
        if (per_point) U3[3 * (i / d) + i % d] = U_n[i];
        else U3[i] = U_n[i];
    }
    if (c->ng > 0)
        HIPCHK(c, hipMemcpyAsync(c->Ubuf, U3.data(), U3.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    return NM_OK;
}

static int step_impl(nm_ctx* c, const double* U_n, int per_point, nm_step_stats* st)
{
    hipStream_t s = c->stream;
    const long n = 3 * c->N;
    const int d = c->dim;
    std::vector<double> U3;
    CHK(upload_U(c, U_n, per_point, U3));
    auto t0 = std::chrono::steady_clock::now();
    // predictor and right-hand side, eq. (Fourier_ND_b) (already formed by the previous
    // step's corrector unless the state or b changed since)
    const bool inc_ok = c->pred_ready;
    const bool sfeat_ok = c->pred_ready && c->sfeat_ready;
    c->sfeat_ready = false;
    if (!c->pred_ready)
        LCHK(c, launch_predictor(c->u, c->v, c->a, c->ut, c->b, c->phase, c->rho64, c->damp64, c->N, 3, c->dt, c->beta,
                             c->gam, s));
    c->pred_ready = false;
    c->d32_is_x = false;
    // initial guess
    double t_warm = 0;
    switch (c->opt.warm_start) {
    case NM_WS_COLD: LCHK(c, launch_fill<double>(c->w, 0.0, n, s)); break;
    case NM_WS_TAYLOR: LCHK(c, launch_taylor(c->w, c->u, c->v, c->a, n, c->dt, s)); break;
    case NM_WS_LEARNED: {
        if (!c->net) return fail(c, NM_EINVAL, "learned warm start requested but no network is attached");
        if (!c->ev_warm[0]) {
            HIPCHK(c, hipEventCreate(&c->ev_warm[0]));
            HIPCHK(c, hipEventCreate(&c->ev_warm[1]));
        }
        HIPCHK(c, hipEventRecord(c->ev_warm[0], s));
        nm::WarmArgs wa = warm_args(c);
        if (inc_ok) {
            // the corrector of the previous step already summed |u~ - u_n|^2
            wa.inc = c->winc;
            wa.inc_nb = corrector_blocks(c->N);
        }
        wa.sfeat = c->sfeat;
        wa.sfeat_ready = sfeat_ok;
        if (c->opt.precision == NM_PREC_MIXED) {
            // the first refinement sweep starts from the FP32 copy
            wa.x0f = c->d32;
            c->d32_is_x = true;
        }
        int e = nm::warm_predict(c->net, wa, c->w, s);
        if (e) return fail(c, e == -1 ? NM_EUNSUPPORTED : NM_EHIP, "warm-start network failed");
        HIPCHK(c, hipEventRecord(c->ev_warm[1], s)); // read after the step's final synchronization
        t_warm = -1;
        break;
    }
    default: LCHK(c, launch_copy<double>(c->w, c->u, n, s)); break;
    }
    nm_step_stats local{};
    local.iters[1] = 0;
    if (c->route == NM_ROUTE_GREEN && c->ng > 0) {
        const int nd = (int)(d * c->ng);
        double bn;
        CHK(norm2<double>(c, c->b, &bn));
        PcgResult r1, r2;
        c->green_sweeps = c->green_inner = 0;
        // (a learned iterate further from the solution than zero is replaced by zero)
        CHK(green_solve(c, c->b, c->w, std::sqrt(bn), c->opt.tol, false, &r1, c->opt.warm_start == NM_WS_LEARNED));
        // V = U - u_b on Gamma ; F = G^-1 V / (beta dt^2)   (eqs. Vt, L-determination_ND), on
        // the device: Fdev holds V, then F (d per point), gbuf the force with 3 components
        LCHK(c, launch_gather_gamma(c->gbuf, c->w, c->gidx, c->ng, 3, c->N, s));
        LCHK(c, launch_green_rhs(c->Fdev, c->gbuf, c->Ubuf, per_point, c->ng, d, s));
        LCHK(c, lu_solve_device(c->Gdev, nd, c->permdev, c->dinvdev, c->Fdev, c->luwork, s));
        LCHK(c, launch_green_force(c->gbuf, c->Fdev, 1.0 / c->sp.bdt2, c->ng, d, s));
        // f = F on Gamma (reuse b, no longer needed) ; A u_f = f from the previous u_f
        LCHK(c, launch_fill<double>(c->b, 0.0, n, s));
        LCHK(c, launch_set_gamma(c->b, c->gidx, c->ng, c->gbuf, 1, 3, c->N, s));
        double fn;
        CHK(norm2<double>(c, c->b, &fn));
        CHK(green_solve(c, c->b, c->uf, std::sqrt(fn), c->opt.tol, false, &r2));
        // u_n = u_b + beta dt^2 u_f   (eq. Sol_Real_ND)
        LCHK(c, launch_axpby<double>(c->w, c->w, c->uf, c->sp.bdt2, n, s));
        local.iters[0] = r1.iters;
        local.iters[1] = r2.iters;
        local.sweeps = c->green_sweeps;
        local.inner_iters = c->green_inner;
        // (a zero right-hand side, as at the first step from rest, is solved exactly)
        local.relres = bn > 0 ? std::sqrt(r1.rr / bn) : 0.0;
        local.relres0 = bn > 0 ? std::sqrt(r1.rr0 / bn) : 0.0;
        c->F_on_device = true;
    } else {
        if (c->ng > 0) LCHK(c, launch_set_gamma(c->w, c->gidx, c->ng, c->Ubuf, per_point, 3, c->N, s));
        if (c->ng > 0 && c->d32_is_x)
            LCHK(c, launch_set_gamma_f32(c->d32, c->gidx, c->ng, c->Ubuf, per_point, 3, c->N, s));
        // reference residual r_bar = P (b - A u_bar) (left in c->r); from the lifting
        // responses when U is uniform on Gamma
        double bref;
        if (c->lift && !per_point) CHK(lift_bref(c, U3.data(), &bref));
        else CHK(projected_bref(c, c->w, &bref));
        // the zero start is u_bar itself, so its initial residual is r_bar
        double rr0 = c->opt.warm_start == NM_WS_COLD ? bref * bref : -1.0;
        // a learned iterate whose residual exceeds the zero start's is replaced by the zero
        // start (u_bar, residual r_bar), so the learned start never begins further away
        const bool guard = c->opt.warm_start == NM_WS_LEARNED;
        auto restart_from_zero = [&]() -> int {
            LCHK(c, launch_fill<double>(c->w, 0.0, n, s));
            if (c->ng > 0) LCHK(c, launch_set_gamma(c->w, c->gidx, c->ng, c->Ubuf, per_point, 3, c->N, s));
            c->d32_is_x = false;
            if (c->lift && !per_point) CHK(lift_bref(c, U3.data(), &bref));
            else CHK(projected_bref(c, c->w, &bref));
            rr0 = bref * bref;
            c->ws_rejected++;
            return NM_OK;
        };
        if (c->opt.precision == NM_PREC_MIXED) {
            bool rejected = false;
            CHK(solve_mixed(c, c->w, bref, &local, rr0, guard ? &rejected : nullptr));
            if (rejected) {
                CHK(restart_from_zero());
                CHK(solve_mixed(c, c->w, bref, &local, rr0));
            }
            if (c->opt.true_residual) {
                CHK(apply_A<double>(c, c->w, c->q, c->mask));
                LCHK(c, launch_residual<double>(c->b, c->q, c->r, c->mask, c->N, 3, c->part_a, s));
                LCHK(c, launch_reduce(c->part_a, vec_blocks(n), c->scal, RED_STORE_RR, 0, s));
                CHK(read_scalars(c));
                local.relres = std::sqrt(c->hscal[S_RR]) / (bref > 0 ? bref : 1.0);
            }
        } else {
            if (guard) {
                // residual of the learned iterate, kept in c->r for the solve unless rejected
                CHK(apply_A<double>(c, c->w, c->q, c->mask));
                LCHK(c, launch_residual<double>(c->b, c->q, c->r, c->mask, c->N, 3, c->part_a, s));
                LCHK(c, launch_reduce(c->part_a, vec_blocks(n), c->scal, RED_STORE_RR, 0, s));
                CHK(read_scalars(c));
                rr0 = c->hscal[S_RR];
                if (rr0 > bref * bref) CHK(restart_from_zero());
            }
            PcgResult r1;
            CHK(pcg<double>(c, c->b, c->w, c->r, c->p, c->q, true, false, bref, c->opt.tol, c->opt.max_iter,
                            -1, false, &r1, rr0));
            local.iters[0] = r1.iters;
            local.relres = std::sqrt(r1.rr) / (bref > 0 ? bref : 1.0);
            local.relres0 = std::sqrt(r1.rr0) / (bref > 0 ? bref : 1.0);
            if (c->opt.true_residual) {
                CHK(apply_A<double>(c, c->w, c->q, c->mask));
                LCHK(c, launch_residual<double>(c->b, c->q, c->r, c->mask, c->N, 3, c->part_a, s));
                LCHK(c, launch_reduce(c->part_a, vec_blocks(n), c->scal, RED_STORE_RR, 0, s));
                CHK(read_scalars(c));
                local.relres = std::sqrt(c->hscal[S_RR]) / (bref > 0 ? bref : 1.0);
            }
        }
        if (c->opt.compute_reaction && c->ng > 0) {
            // F = (A u - b)|Gamma / (beta dt^2)
            CHK(apply_A<double>(c, c->w, c->q, nullptr));
            LCHK(c, launch_axpby<double>(c->r, c->q, c->b, -1.0, n, s));
            LCHK(c, launch_gather_gamma(c->gbuf, c->r, c->gidx, c->ng, 3, c->N, s));
            std::vector<double> g3(3 * c->ng);
            HIPCHK(c, hipMemcpyAsync(g3.data(), c->gbuf, g3.size() * sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(c, hipStreamSynchronize(s));
            for (long pnt = 0; pnt < c->ng; pnt++)
                for (int j = 0; j < d; j++) c->F_last[d * pnt + j] = g3[3 * pnt + j] / c->sp.bdt2;
        }
    }
    // corrector, fused with the predictor and right-hand side of the next step; then
    // u <- u_n (pointer swap)
    // with the learned start the corrector also leaves the next step's state features
    uint16_t* sf = (c->opt.warm_start == NM_WS_LEARNED && c->net && c->sfeat) ? c->sfeat : nullptr;
    LCHK(c, launch_corrector_predictor(c->w, c->ut, c->v, c->a, c->b, c->phase, c->rho64, c->damp64, c->N, 3, c->dt,
                                       c->beta, c->gam, c->winc, sf, s));
    c->sfeat_ready = sf != nullptr;
    std::swap(c->u, c->w);
    HIPCHK(c, hipStreamSynchronize(s));
    c->pred_ready = true;
    c->step++;
    local.t_step_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (t_warm < 0) {
        float ms = 0;
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev_warm[0], c->ev_warm[1]));
        t_warm = ms;
    }
    local.t_warm_ms = t_warm;
    if (st) *st = local;
    return NM_OK;
}

int nm_newmark_step(nm_ctx* c, const double* U_n, int per_point, nm_step_stats* st)
{
    if (!c) return NM_EINVAL;
    if (c->explicit_scheme)
        return fail(c, NM_EINVAL, "this context runs the explicit scheme (beta = 0): call nm_explicit_step");
    return step_impl(c, U_n, per_point, st);
}

// n_steps central-difference steps (section 2.3) without a host round trip in between.
static int explicit_impl(nm_ctx* c, const double* Udot, int per_point, int n_steps, nm_step_stats* st)
{
    hipStream_t s = c->stream;
    const int d = c->dim;
    const long row = c->ng > 0 ? (per_point ? (long)d * c->ng : d) : 0;
    const size_t total = (size_t)row * n_steps;
    if (c->ng > 0) {
        if (!Udot) return fail(c, NM_EINVAL, "null prescribed velocity");
        for (size_t i = 0; i < total; i++)
            if (!std::isfinite(Udot[i])) return fail(c, NM_ENAN, "non-finite prescribed velocity");
        if (total > c->ubatch_cap) {
            // grown on demand; released with the context
            double* nb = nullptr;
            CHK(dalloc(c, &nb, total));
            c->ubatch = nb;
            c->ubatch_cap = total;
        }
        HIPCHK(c, hipMemcpyAsync(c->ubatch, Udot, total * sizeof(double), hipMemcpyHostToDevice, s));
    }
    auto t0 = std::chrono::steady_clock::now();
    const double dt = c->dt;
    for (int k = 0; k < n_steps; k++) {
        // u_n = u + dt v + dt^2/2 a, and its x spectrum
        XFwdArgs fa = xf_args(c, c->spec64);
        fa.u = c->u;
        fa.v = c->v;
        fa.a = c->a;
        fa.dt = dt;
        LCHK(c, launch_xfwd<double>(XF_EXPLICIT, c->n1, fa, c->tw64, s));
        // (dt/2) div sigma(u_n) -> v <- v + dt/2 a + (dt/2) div sigma / rho, a <- div sigma / rho
        XInvArgs ia = xi_args(c, c->spec64, nullptr, nullptr, c->rho64, nullptr, nullptr);
        ia.p = c->v;
        ia.x = c->a;
        ia.dt = dt;
        CHK(chain_operator_rest<double>(c, ia, XI_EXPLICIT, -0.5 * dt));
        // Gamma: the force that gives the prescribed velocity
        if (c->ng > 0)
            LCHK(c, launch_explicit_gamma(c->v, c->a, c->phase, c->rho64, c->gidx, c->ng, c->ubatch + (size_t)row * k,
                                          per_point, d, c->N, dt, c->Fdev, s));
    }
    HIPCHK(c, hipStreamSynchronize(s));
    c->step += n_steps;
    c->F_on_device = c->ng > 0;
    if (st) {
        nm_step_stats local{};
        local.t_step_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() / n_steps;
        *st = local;
    }
    return NM_OK;
}

int nm_explicit_step(nm_ctx* c, const double* Udot, int per_point, int n_steps, nm_step_stats* st)
{
    if (!c) return NM_EINVAL;
    if (!c->explicit_scheme)
        return fail(c, NM_EINVAL, "nm_explicit_step needs a context created with beta = 0 (central differences)");
    if (n_steps < 1) return fail(c, NM_EINVAL, "n_steps must be positive");
    return explicit_impl(c, Udot, per_point, n_steps, st);
}

int nm_omega2_max(nm_ctx* c, void* x_dev, int iters, double* omega2)
{
    if (!c) return NM_EINVAL;
    if (!x_dev || iters < 0 || !omega2) return fail(c, NM_EINVAL, "bad arguments");
    hipStream_t s = c->stream;
    double* x = (double*)x_dev;
    double* y = c->q;
    const long n = 3 * c->N;
    c->pred_ready = false; // the work field q is shared with the step
    double lam = 0.0;
    for (int it = 0; it <= iters; it++) {
        // x <- x / |x|_rho
        LCHK(c, launch_rho_norm2(x, c->phase, c->rhot64, c->N, c->part_a, s));
        LCHK(c, launch_reduce(c->part_a, vec_blocks(n), c->scal, RED_STORE_SLOT, 6, s));
        CHK(read_scalars(c));
        const double m = c->hscal[6];
        if (!(m > 0) || !std::isfinite(m)) return fail(c, NM_ENAN, "start vector has no rho-weighted norm");
        LCHK(c, launch_axpby<double>(x, x, x, 1.0 / std::sqrt(m) - 1.0, n, s));
        // y = K x = -div sigma(x) ; lam = x . y
        CHK(div_stress(c, x, y, -1.0));
        CHK(dot64(c, x, y, &lam));
        if (it == iters) break;
        // x <- rho^-1 K x
        LCHK(c, launch_div_rho(x, y, c->phase, c->rhot64, c->N, s));
    }
    HIPCHK(c, hipStreamSynchronize(s));
    *omega2 = lam;
    return NM_OK;
}

int nm_apply_operator(nm_ctx* c, const void* u_dev, void* Au_dev, int dtype)
{
    if (!c) return NM_EINVAL;
    if (!u_dev || !Au_dev || u_dev == Au_dev) return fail(c, NM_EINVAL, "bad buffers");
    if (dtype == NM_FP64) return apply_A<double>(c, (const double*)u_dev, (double*)Au_dev, nullptr);
    if (dtype == NM_FP32 && !c->spec32) return fail(c, NM_EINVAL, "FP32 buffers are not held by an explicit context");
    if (dtype == NM_FP32) return apply_A<float>(c, (const float*)u_dev, (float*)Au_dev, nullptr);
    return fail(c, NM_EINVAL, "dtype must be NM_FP64 or NM_FP32");
}

int nm_precond_apply(nm_ctx* c, const void* r_dev, void* z_dev, int dtype)
{
    if (!c) return NM_EINVAL;
    if (c->explicit_scheme) return fail(c, NM_EINVAL, "the explicit scheme has no preconditioner");
    if (!r_dev || !z_dev || r_dev == z_dev) return fail(c, NM_EINVAL, "bad buffers");
    if (dtype == NM_FP64) return precond_impl<double>(c, (const double*)r_dev, (double*)z_dev);
    if (dtype == NM_FP32) return precond_impl<float>(c, (const float*)r_dev, (float*)z_dev);
    return fail(c, NM_EINVAL, "dtype must be NM_FP64 or NM_FP32");
}

int nm_pcg_solve(nm_ctx* c, const void* b_dev, void* x_dev, int masked, double tol, int max_iter, int fixed_iters,
                 int* iters, double* relres)
{
    if (!c) return NM_EINVAL;
    if (c->explicit_scheme) return fail(c, NM_EINVAL, "the explicit scheme has no Krylov solver");
    if (!b_dev || !x_dev || b_dev == x_dev) return fail(c, NM_EINVAL, "bad buffers");
    if (!(tol > 0) || max_iter <= 0) return fail(c, NM_EINVAL, "bad tolerance or max_iter");
    double bref;
    // the projected reference norm reads c->b, so stage the right-hand side there
    c->pred_ready = false;
    HIPCHK(c, hipMemcpyAsync(c->b, b_dev, 3 * c->N * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    if (masked) {
        CHK(projected_bref(c, (const double*)x_dev, &bref));
    } else {
        double bn;
        CHK(norm2<double>(c, c->b, &bn));
        bref = std::sqrt(bn);
    }
    PcgResult pr;
    CHK(pcg<double>(c, c->b, (double*)x_dev, c->r, c->p, c->q, masked != 0, false, bref, tol, max_iter,
                    fixed_iters, false, &pr));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (iters) *iters = pr.iters;
    if (relres) *relres = std::sqrt(pr.rr) / (bref > 0 ? bref : 1.0);
    return NM_OK;
}

int nm_get_state(const nm_ctx* cc, double* u, double* v, double* a, double* F_gamma, int64_t* step)
{
    nm_ctx* c = const_cast<nm_ctx*>(cc);
    if (!c) return NM_EINVAL;
    const size_t bytes = c->dim * c->N * sizeof(double);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (c->F_on_device) {
        HIPCHK(c, hipMemcpy(c->F_last.data(), c->Fdev, c->F_last.size() * sizeof(double), hipMemcpyDeviceToHost));
        c->F_on_device = false;
    }
    if (u) HIPCHK(c, hipMemcpy(u, c->u, bytes, hipMemcpyDeviceToHost));
    if (v) HIPCHK(c, hipMemcpy(v, c->v, bytes, hipMemcpyDeviceToHost));
    if (a) HIPCHK(c, hipMemcpy(a, c->a, bytes, hipMemcpyDeviceToHost));
    if (F_gamma && !c->F_last.empty()) std::memcpy(F_gamma, c->F_last.data(), c->F_last.size() * sizeof(double));
    if (step) *step = c->step;
    return NM_OK;
}

int nm_set_state(nm_ctx* c, const double* u, const double* v, const double* a, int64_t step)
{
    if (!c) return NM_EINVAL;
    if (!u || !v || !a) return fail(c, NM_EINVAL, "u, v and a are required");
    const size_t bytes = c->dim * c->N * sizeof(double);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(c->u, u, bytes, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->v, v, bytes, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->a, a, bytes, hipMemcpyHostToDevice));
    c->step = step;
    c->pred_ready = false;
    return NM_OK;
}

int nm_state_device_ptrs(nm_ctx* c, void** u, void** v, void** a)
{
    if (!c) return NM_EINVAL;
    c->pred_ready = false; // the caller may write the state through these views
    if (u) *u = c->u;
    if (v) *v = c->v;
    if (a) *a = c->a;
    return NM_OK;
}

int nm_profile_passes(nm_ctx* c, int which, const void* u_dev, void* out_dev, int dtype, int reps, double* ms)
{
    if (!c) return NM_EINVAL;
    if (!u_dev || !out_dev || u_dev == out_dev || !ms || reps <= 0 || (which != 0 && which != 1))
        return fail(c, NM_EINVAL, "bad arguments");
    if (c->explicit_scheme && (which == 1 || dtype != NM_FP64))
        return fail(c, NM_EINVAL, "an explicit context profiles the FP64 operator only");
    if (dtype == NM_FP64) return profile_impl<double>(c, which, (const double*)u_dev, (double*)out_dev, reps, ms);
    if (dtype == NM_FP32) return profile_impl<float>(c, which, (const float*)u_dev, (float*)out_dev, reps, ms);
    return fail(c, NM_EINVAL, "dtype must be NM_FP64 or NM_FP32");
}

int nm_ws_attach(nm_ctx* c, nm_net* net)
{
    if (!c) return NM_EINVAL;
    if (c->explicit_scheme && net) return fail(c, NM_EINVAL, "the explicit scheme has no initial iterate to predict");
    if (net != c->net) c->l0mat_version = 0; // versions of different networks are unrelated
    c->net = net;
    if (!net || c->feat) return NM_OK;
    CHK(dalloc(c, &c->feat, 32 * (size_t)c->N));
    CHK(dalloc(c, &c->sfeat, 16 * (size_t)c->N));
    CHK(dalloc(c, &c->matf, 22 * (size_t)c->nph));
    CHK(dalloc(c, &c->wscale, 1));
    CHK(dalloc(c, &c->wred, 512));
    CHK(dalloc(c, &c->l0mat, 16 * (size_t)c->N));
    std::vector<double> C(21 * (size_t)c->nph), rho(c->nph);
    HIPCHK(c, hipMemcpy(C.data(), c->C64, C.size() * sizeof(double), hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(rho.data(), c->rho64, rho.size() * sizeof(double), hipMemcpyDeviceToHost));
    std::vector<float> mf(22 * (size_t)c->nph);
    const double c11 = c->sp.Cbar[0] > 0 ? c->sp.Cbar[0] : 1.0;
    for (int g = 0; g < c->nph; g++) {
        mf[22 * g] = (float)(rho[g] / c->sp.rhobar);
        for (int k = 0; k < 21; k++) mf[22 * g + 1 + k] = (float)(C[21 * g + k] / c11);
    }
    HIPCHK(c, hipMemcpy(c->matf, mf.data(), mf.size() * sizeof(float), hipMemcpyHostToDevice));
    return NM_OK;
}

int nm_ws_features(nm_ctx* c, void* feat_dev)
{
    if (!c || !c->feat) return fail(c, NM_EINVAL, "call nm_ws_attach first");
    hipStream_t s = c->stream;
    // predictor of the next step (the step recomputes the same values)
    LCHK(c, launch_predictor(c->u, c->v, c->a, c->ut, c->b, c->phase, c->rho64, c->damp64, c->N, 3, c->dt, c->beta,
                             c->gam, s));
    nm::WarmArgs a = warm_args(c);
    if (feat_dev) a.feat = (uint16_t*)feat_dev;
    LCHK(c, nm::warm_features(a, s));
    HIPCHK(c, hipStreamSynchronize(s));
    return NM_OK;
}

int nm_ws_predict(nm_ctx* c, void* x0_dev)
{
    if (!c || !c->net || !x0_dev) return fail(c, NM_EINVAL, "attach a network and pass x0");
    hipStream_t s = c->stream;
    LCHK(c, launch_predictor(c->u, c->v, c->a, c->ut, c->b, c->phase, c->rho64, c->damp64, c->N, 3, c->dt, c->beta,
                             c->gam, s));
    int e = nm::warm_predict(c->net, warm_args(c), (double*)x0_dev, s);
    if (e) return fail(c, e == -1 ? NM_EUNSUPPORTED : NM_EHIP, "warm-start network failed");
    HIPCHK(c, hipStreamSynchronize(s));
    return NM_OK;
}

int nm_ws_target(nm_ctx* c, void* target_dev)
{
    if (!c || !c->feat || !target_dev) return fail(c, NM_EINVAL, "call nm_ws_attach first");
    LCHK(c, nm::warm_target(warm_args(c), c->a, c->sp.bdt2, (float*)target_dev, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return NM_OK;
}

int nm_ws_residual_sample(nm_ctx* c, const double* U_next, int per_point, void* feat_dev, void* rp_dev, double* s_out,
                          double* cref_out, double* crefM_out)
{
    if (!c || !c->feat || !feat_dev || !rp_dev || !s_out || !cref_out)
        return fail(c, NM_EINVAL, "call nm_ws_attach first and pass every output");
    if (c->route == NM_ROUTE_GREEN) return fail(c, NM_EINVAL, "residual samples need the projected route");
    hipStream_t s = c->stream;
    const long n = 3 * c->N;
    std::vector<double> U3;
    CHK(upload_U(c, U_next, per_point, U3));
    // predictor, b = rho u~, features and scale of the coming step
    LCHK(c, launch_predictor(c->u, c->v, c->a, c->ut, c->b, c->phase, c->rho64, c->damp64, c->N, 3, c->dt, c->beta,
                             c->gam, s));
    nm::WarmArgs a = warm_args(c);
    a.feat = (uint16_t*)feat_dev;
    LCHK(c, nm::warm_features(a, s));
    // rp = P (b - A u~_Gamma), u~_Gamma = u~ with U(t_{n+1}) on Gamma
    double* rp = (double*)rp_dev;
    LCHK(c, launch_copy<double>(c->w, c->ut, n, s));
    if (c->ng > 0) LCHK(c, launch_set_gamma(c->w, c->gidx, c->ng, c->Ubuf, per_point, 3, c->N, s));
    CHK(apply_A<double>(c, c->w, c->q, c->mask));
    LCHK(c, launch_residual<double>(c->b, c->q, rp, c->mask, c->N, 3, c->part_a, s));
    double bref;
    CHK(projected_bref(c, c->w, &bref)); // leaves r_bar = P (b - A u_bar) in c->r
    if (crefM_out) {
        CHK(precond_masked(c, c->r, c->z));
        CHK(dot64(c, c->r, c->z, crefM_out));
    }
    HIPCHK(c, hipMemcpyAsync(s_out, c->wscale, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    *cref_out = bref * bref;
    return NM_OK;
}

int nm_ws_train_residual(nm_ctx* c, const void* feat_dev, const void* rp_dev, double scale, double cref, int metric,
                         float lr, float* loss)
{
    if (!c || !c->net || !feat_dev || !rp_dev || !(lr > 0) || !(cref > 0) || !std::isfinite(scale) ||
        (metric != 0 && metric != 1))
        return fail(c, NM_EINVAL, "bad arguments (attached network, buffers, metric 0/1, lr > 0, cref > 0)");
    hipStream_t s = c->stream;
    const long n = 3 * c->N;
    const uint16_t* feat = (const uint16_t*)feat_dev;
    nm::WarmArgs a = warm_args(c);
    // y = s P net(f) ; q = P A y ; r0 = rp - q
    int e = nm::warm_residual_forward(c->net, a, feat, scale, c->mask, c->p, s);
    if (e) return fail(c, e == -1 ? NM_EUNSUPPORTED : NM_EHIP, "warm-start network forward failed");
    CHK(apply_A<double>(c, c->p, c->q, c->mask));
    LCHK(c, launch_axpby<double>(c->r, (const double*)rp_dev, c->q, -1.0, n, s));
    double val;
    const double* wvec = c->r; // the vector the loss gradient pulls back through P A P
    if (metric == 0) {
        // L = r0 . r0 / cref
        CHK(norm2<double>(c, c->r, &val));
    } else {
        // L = r0 . (P M P r0) / cref
        CHK(precond_masked(c, c->r, c->w));
        CHK(dot64(c, c->r, c->w, &val));
        wvec = c->w;
    }
    // dL/dpred = -2 s P A (r0 or P M P r0) / cref  (A and M symmetric)
    CHK(apply_A<double>(c, wvec, c->z, c->mask));
    e = nm::warm_residual_backward(c->net, a, feat, c->z, -2.0 * scale / cref, lr, s);
    if (e) return fail(c, NM_EHIP, "warm-start network backward failed");
    HIPCHK(c, hipStreamSynchronize(s));
    if (loss) *loss = (float)(val / cref);
    return NM_OK;
}

void* nm_get_stream(nm_ctx* c) { return c ? (void*)c->stream : nullptr; }

int nm_green_solve(nm_ctx* c, const double* V, double* X)
{
    if (!c) return NM_EINVAL;
    if (!c->Gdev || !V || !X) return fail(c, NM_EINVAL, "no Green matrix in this context, or null vectors");
    const long nd = (long)c->dim * c->ng;
    double* buf = nullptr;
    CHK(dalloc(c, &buf, nd));
    HIPCHK(c, hipMemcpyAsync(buf, V, nd * sizeof(double), hipMemcpyHostToDevice, c->stream));
    LCHK(c, lu_solve_device(c->Gdev, (int)nd, c->permdev, c->dinvdev, buf, c->luwork, c->stream));
    HIPCHK(c, hipMemcpyAsync(X, buf, nd * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->allocs.erase(std::find(c->allocs.begin(), c->allocs.end(), (void*)buf));
    HIPCHK(c, hipFree(buf));
    return NM_OK;
}

int nm_green_matrix(const nm_ctx* c, double* G)
{
    if (!c || !G) return NM_EINVAL;
    if (c->G.empty()) return NM_EINVAL;
    std::memcpy(G, c->G.data(), c->G.size() * sizeof(double));
    return NM_OK;
}

} // extern "C"
