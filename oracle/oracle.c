/*
 * Plain FP64 CPU oracle for the implicit FFT-based Newmark solver of
 * Sancho, Rey de Pedraza, Lafourcade, Lebensohn and Segurado,
 * "An implicit FFT-based method for wave propagation in elastic
 * heterogeneous media" (arXiv 2211.08263).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link
 * or call this file; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code with the GPU
 * library.
 *
 * Everything is single threaded, double precision, written for checking by
 * eye rather than for speed:
 *   - its own iterative radix-2 complex FFT (unnormalized forward, inverse
 *     divided by the number of points);
 *   - the operator of eq. (Fourier_ND_A) with full 4th-order tensors and all
 *     d*d displacement derivatives;
 *   - the reference-medium preconditioner of eqs. (precond), (acous);
 *   - textbook preconditioned conjugate gradients (section 2.2.3);
 *   - the Green-matrix route of eqs. (f_discrete)-(L-determination_ND)
 *     and Algorithm 2, a projected route, and a dense direct solve;
 *   - Newmark beta/gamma (eq. Newmark);
 *   - a direct 3x3x3 periodic convolution with forward and backward passes
 *     (learned warm start).
 *
 * Readings of the paper taken here (where it is silent or garbled):
 *   - discrete frequencies in standard DFT order, xi_k = 2 pi k / L for
 *     k < N/2, 2 pi (k - N) / L for k > N/2 and xi = 0 at k = N/2;
 *   - Krylov vectors live in real space; stopping rule ||r|| <= tol ||b||
 *     on the recursively updated residual;
 *   - G[d q + i][d p + j] = u^i_(p,j)(x_q), so that u_Gamma = G F;
 *   - a force at a Gamma voxel is the nodal value F (no 1/h^d);
 *   - initial acceleration a0 = div(C : grad^s u0) / rho.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* ------------------------------------------------------------------------- */
/* Radix-2 FFT (Cooley-Tukey, decimation in time, bit-reversed input)        */
/* ------------------------------------------------------------------------- */

/* In-place length-n transform; sign = -1 forward (e^{-2 pi i nk/N}),
 * +1 inverse (unnormalized).  n must be a power of two. */
static void fft1d(cplx *a, int n, int sign)
{
    for (int i = 1, j = 0; i < n; i++) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1)
            j ^= bit;
        j ^= bit;
        if (i < j) {
            cplx t = a[i];
            a[i] = a[j];
            a[j] = t;
        }
    }
    for (int len = 2; len <= n; len <<= 1) {
        int half = len / 2;
        for (int k = 0; k < half; k++) {
            double ang = sign * 2.0 * M_PI * (double)k / (double)len;
            cplx w = cos(ang) + I * sin(ang);
            for (int i = 0; i < n; i += len) {
                cplx u = a[i + k];
                cplx v = a[i + k + half] * w;
                a[i + k] = u + v;
                a[i + k + half] = u - v;
            }
        }
    }
}

/* Multi-dimensional transform of an array with axis 0 fastest (n[0]),
 * applied axis by axis. */
void or_fftn(cplx *a, int d, const int *n, int sign)
{
    int N[3] = {1, 1, 1};
    for (int i = 0; i < d; i++)
        N[i] = n[i];
    long total = (long)N[0] * N[1] * N[2];
    int maxn = N[0] > N[1] ? N[0] : N[1];
    maxn = maxn > N[2] ? maxn : N[2];
    cplx *line = malloc(sizeof(cplx) * maxn);
    long stride[3] = {1, N[0], (long)N[0] * N[1]};
    for (int ax = 0; ax < 3; ax++) {
        int len = N[ax];
        if (len == 1)
            continue;
        long st = stride[ax];
        for (long base = 0; base < total; base++) {
            /* base must have coordinate 0 along ax */
            long c = (base / st) % len;
            if (c != 0)
                continue;
            for (int m = 0; m < len; m++)
                line[m] = a[base + m * st];
            fft1d(line, len, sign);
            for (int m = 0; m < len; m++)
                a[base + m * st] = line[m];
        }
    }
    free(line);
}

/* Frequency of DFT index k on an axis of n points and length L. */
double or_xi(int k, int n, double L)
{
    if (n == 1)
        return 0.0;
    if (2 * k == n)
        return 0.0; /* Nyquist bin: zero (keeps the operator real and symmetric) */
    int kk = (2 * k < n) ? k : k - n;
    return 2.0 * M_PI * (double)kk / L;
}

/* ------------------------------------------------------------------------- */
/* Problem description                                                        */
/* ------------------------------------------------------------------------- */
typedef struct {
    int d;                 /* 1, 2 or 3 */
    int n[3];              /* points per axis, axis 0 fastest; n[i] = 1 for i >= d */
    double L[3];           /* box lengths */
    int n_phases;
    const uint16_t *phase; /* per voxel */
    const double *C21;     /* per phase: upper triangle of the Voigt 6x6 */
    const double *rho;     /* per phase */
    double dt, beta, gamma_nm;
    const double *damp;    /* per phase viscous coefficient c (force -c v), or NULL for none */
    int diff_rule;         /* 0 spectral derivative, 1 and 2 centred differences (or_xi_rule) */
} or_prob;

/* Density seen by the implicit operator: rho + gamma dt c (the viscous term of
 * M a + C v + K u = f folded in by the Newmark update v_n = v~ + gamma dt a_n). */
static double rho_op(const or_prob *p, int g)
{
    return p->rho[g] + (p->damp ? p->gamma_nm * p->dt * p->damp[g] : 0.0);
}

/* Voigt index of the symmetric pair (i, j): 11,22,33,23,13,12. */
static int voigt_index(int i, int j)
{
    if (i == j)
        return i;
    int s = i + j;
    return s == 3 ? 3 : (s == 2 ? 4 : 5); /* (1,2)->3  (0,2)->4  (0,1)->5 */
}

static double voigt_entry(const double *c21, int a, int b)
{
    if (a > b) {
        int t = a;
        a = b;
        b = t;
    }
    /* row-major upper triangle offset */
    int off = a * 6 - a * (a - 1) / 2;
    return c21[off + (b - a)];
}

/* Full tensor C_ijkl of one phase (engineering-shear Voigt => no factors). */
static void tensor_of_phase(const double *c21, double C[3][3][3][3])
{
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            for (int k = 0; k < 3; k++)
                for (int l = 0; l < 3; l++)
                    C[i][j][k][l] = voigt_entry(c21, voigt_index(i, j), voigt_index(k, l));
}

static long nvox(const or_prob *p) { return (long)p->n[0] * p->n[1] * p->n[2]; }

/* The frequency a differentiation rule puts in place of xi (section 5 proposes discrete
 * finite-difference rules against the noise of high contrast):
 *   0: the spectral derivative, symbol i xi (Nyquist bin zero, as above);
 *   1: the centred difference (f(x + h) - f(x - h)) / (2h), symbol i sin(xi h) / h;
 *   2: the fourth-order centred difference
 *      (-f(x + 2h) + 8 f(x + h) - 8 f(x - h) + f(x - 2h)) / (12 h),
 *      symbol i (8 sin(xi h) - sin(2 xi h)) / (6 h).
 * Both difference symbols vanish at the Nyquist bin by themselves. */
double or_xi_rule(int k, int n, double L, int rule)
{
    double xi = or_xi(k, n, L);
    if (rule == 0 || n == 1)
        return xi;
    double h = L / n;
    if (rule == 1)
        return sin(xi * h) / h;
    return (8.0 * sin(xi * h) - sin(2.0 * xi * h)) / (6.0 * h);
}

static void freq_of(const or_prob *p, long idx, double xi[3])
{
    int k0 = (int)(idx % p->n[0]);
    int k1 = (int)((idx / p->n[0]) % p->n[1]);
    int k2 = (int)(idx / ((long)p->n[0] * p->n[1]));
    xi[0] = or_xi_rule(k0, p->n[0], p->L[0], p->diff_rule);
    xi[1] = or_xi_rule(k1, p->n[1], p->L[1], p->diff_rule);
    xi[2] = or_xi_rule(k2, p->n[2], p->L[2], p->diff_rule);
}

/* ------------------------------------------------------------------------- */
/* Spectral derivative and the divergence of the stress                       */
/* ------------------------------------------------------------------------- */

/* out = D_k f = IDFT( i xi_k DFT(f) ), real input and output. */
void or_deriv(const or_prob *p, const double *f, int k, double *out)
{
    long N = nvox(p);
    cplx *a = malloc(sizeof(cplx) * N);
    for (long v = 0; v < N; v++)
        a[v] = f[v];
    or_fftn(a, 3, p->n, -1);
    for (long v = 0; v < N; v++) {
        double xi[3];
        freq_of(p, v, xi);
        a[v] *= I * xi[k];
    }
    or_fftn(a, 3, p->n, +1);
    for (long v = 0; v < N; v++)
        out[v] = creal(a[v]) / (double)N;
    free(a);
}

/* Stress sigma_jk(x) = C_jklm(x) eps_lm(x), eps_lm = (D_m u_l + D_l u_m)/2.
 * sig is d*d fields (row major j,k). */
void or_stress(const or_prob *p, const double *u, double *sig)
{
    int d = p->d;
    long N = nvox(p);
    double *Du = malloc(sizeof(double) * d * d * N); /* Du[l][m] = D_m u_l */
    for (int l = 0; l < d; l++)
        for (int m = 0; m < d; m++)
            or_deriv(p, u + l * N, m, Du + (l * d + m) * N);
    double (*C)[3][3][3][3] = malloc(sizeof(double) * 81 * p->n_phases);
    for (int g = 0; g < p->n_phases; g++)
        tensor_of_phase(p->C21 + 21 * g, C[g]);
    for (long v = 0; v < N; v++) {
        int g = p->phase[v];
        double eps[3][3];
        for (int l = 0; l < d; l++)
            for (int m = 0; m < d; m++)
                eps[l][m] = 0.5 * (Du[(l * d + m) * N + v] + Du[(m * d + l) * N + v]);
        for (int j = 0; j < d; j++)
            for (int k = 0; k < d; k++) {
                double s = 0.0;
                for (int l = 0; l < d; l++)
                    for (int m = 0; m < d; m++)
                        s += C[g][j][k][l][m] * eps[l][m];
                sig[(j * d + k) * N + v] = s;
            }
    }
    free(C);
    free(Du);
}

/* out_j = sum_k D_k sigma_jk(u)  (the divergence of the stress). */
void or_div_stress(const or_prob *p, const double *u, double *out)
{
    int d = p->d;
    long N = nvox(p);
    double *sig = malloc(sizeof(double) * d * d * N);
    double *tmp = malloc(sizeof(double) * N);
    or_stress(p, u, sig);
    for (int j = 0; j < d; j++) {
        memset(out + j * N, 0, sizeof(double) * N);
        for (int k = 0; k < d; k++) {
            or_deriv(p, sig + (j * d + k) * N, k, tmp);
            for (long v = 0; v < N; v++)
                out[j * N + v] += tmp[v];
        }
    }
    free(tmp);
    free(sig);
}

/* (A u)_j = -beta dt^2 sum_k D_k sigma_jk(u) + rho u_j   (eq. Fourier_ND_A in real space). */
void or_apply(const or_prob *p, const double *u, double *Au)
{
    int d = p->d;
    long N = nvox(p);
    double c = p->beta * p->dt * p->dt;
    or_div_stress(p, u, Au);
    for (int j = 0; j < d; j++)
        for (long v = 0; v < N; v++)
            Au[j * N + v] = -c * Au[j * N + v] + rho_op(p, p->phase[v]) * u[j * N + v];
}

/* ------------------------------------------------------------------------- */
/* Reference-medium preconditioner, eqs. (precond) and (acous)               */
/* ------------------------------------------------------------------------- */

/* Solve the d x d real system A x = b by Gaussian elimination with partial
 * pivoting (b complex: real and imaginary parts share the elimination). */
static void small_solve(int d, double A[3][3], cplx b[3], cplx x[3])
{
    double M[3][3];
    cplx r[3];
    memcpy(M, A, sizeof(M));
    for (int i = 0; i < d; i++)
        r[i] = b[i];
    for (int c = 0; c < d; c++) {
        int piv = c;
        for (int i = c + 1; i < d; i++)
            if (fabs(M[i][c]) > fabs(M[piv][c]))
                piv = i;
        if (piv != c) {
            for (int j = 0; j < d; j++) {
                double t = M[c][j];
                M[c][j] = M[piv][j];
                M[piv][j] = t;
            }
            cplx t = r[c];
            r[c] = r[piv];
            r[piv] = t;
        }
        for (int i = c + 1; i < d; i++) {
            double f = M[i][c] / M[c][c];
            for (int j = c; j < d; j++)
                M[i][j] -= f * M[c][j];
            r[i] -= f * r[c];
        }
    }
    for (int i = d - 1; i >= 0; i--) {
        cplx s = r[i];
        for (int j = i + 1; j < d; j++)
            s -= M[i][j] * x[j];
        x[i] = s / M[i][i];
    }
}

/* Volume averages of the stiffness tensor and the density. */
void or_reference_medium(const or_prob *p, double Cbar[81], double *rhobar)
{
    long N = nvox(p);
    double (*C)[3][3][3][3] = malloc(sizeof(double) * 81 * p->n_phases);
    long *count = calloc(p->n_phases, sizeof(long));
    for (int g = 0; g < p->n_phases; g++)
        tensor_of_phase(p->C21 + 21 * g, C[g]);
    for (long v = 0; v < N; v++)
        count[p->phase[v]]++;
    for (int t = 0; t < 81; t++)
        Cbar[t] = 0.0;
    *rhobar = 0.0;
    for (int g = 0; g < p->n_phases; g++) {
        double w = (double)count[g] / (double)N;
        const double *cg = &C[g][0][0][0][0];
        for (int t = 0; t < 81; t++)
            Cbar[t] += w * cg[t];
        *rhobar += w * rho_op(p, g);
    }
    free(count);
    free(C);
}

/* z = M r: per frequency, solve (beta dt^2 K(xi) + rhobar I) z^ = r^ with
 * K_ij = Cbar_ikjm xi_k xi_m. */
void or_precond(const or_prob *p, const double *r, double *z)
{
    int d = p->d;
    long N = nvox(p);
    double Cbar[81], rhobar;
    or_reference_medium(p, Cbar, &rhobar);
#define CB(i, j, k, l) Cbar[(((i)*3 + (j)) * 3 + (k)) * 3 + (l)]
    double c = p->beta * p->dt * p->dt;
    cplx *a = malloc(sizeof(cplx) * d * N);
    for (int j = 0; j < d; j++) {
        for (long v = 0; v < N; v++)
            a[j * N + v] = r[j * N + v];
        or_fftn(a + j * N, 3, p->n, -1);
    }
    for (long v = 0; v < N; v++) {
        double xi[3], K[3][3];
        freq_of(p, v, xi);
        for (int i = 0; i < d; i++)
            for (int j = 0; j < d; j++) {
                double s = 0.0;
                for (int k = 0; k < d; k++)
                    for (int m = 0; m < d; m++)
                        s += CB(i, k, j, m) * xi[k] * xi[m];
                K[i][j] = c * s + (i == j ? rhobar : 0.0);
            }
        cplx b[3], x[3];
        for (int j = 0; j < d; j++)
            b[j] = a[j * N + v];
        small_solve(d, K, b, x);
        for (int j = 0; j < d; j++)
            a[j * N + v] = x[j];
    }
#undef CB
    for (int j = 0; j < d; j++) {
        or_fftn(a + j * N, 3, p->n, +1);
        for (long v = 0; v < N; v++)
            z[j * N + v] = creal(a[j * N + v]) / (double)N;
    }
    free(a);
}

/* ------------------------------------------------------------------------- */
/* Preconditioned conjugate gradients                                         */
/* ------------------------------------------------------------------------- */
static double dot(const double *a, const double *b, long n)
{
    double s = 0.0;
    for (long i = 0; i < n; i++)
        s += a[i] * b[i];
    return s;
}

static void apply_mask(double *x, const uint8_t *fixed, long n)
{
    if (!fixed)
        return;
    for (long i = 0; i < n; i++)
        if (fixed[i])
            x[i] = 0.0;
}

/*
 * Solve A x = b by PCG from the initial guess in x.  With a mask (fixed[i]
 * != 0 marks a constrained dof) the iteration runs on the free dofs only
 * (operator P A P, preconditioner P M P) and the constrained entries of x
 * are left as given.
 *
 * Stops when ||r|| <= tol * bref (bref > 0), or after exactly fixed_iters
 * iterations when fixed_iters >= 0.  Returns the number of iterations (each
 * iteration is one product A p), or -1 if max_iter was reached without
 * convergence.  *relres receives the final ||r|| / bref of the recursive
 * residual.
 */
int or_pcg(const or_prob *p, const double *b, double *x, const uint8_t *fixed, double bref,
           double tol, int max_iter, int fixed_iters, double *relres)
{
    long n = (long)p->d * nvox(p);
    double *r = malloc(sizeof(double) * n);
    double *z = malloc(sizeof(double) * n);
    double *pp = malloc(sizeof(double) * n);
    double *q = malloc(sizeof(double) * n);
    or_apply(p, x, q);
    for (long i = 0; i < n; i++)
        r[i] = b[i] - q[i];
    apply_mask(r, fixed, n);
    double rr = dot(r, r, n);
    int it = 0, status = 0;
    if (bref <= 0.0)
        bref = 1.0;
    if (fixed_iters < 0 && sqrt(rr) <= tol * bref)
        goto done;
    if (fixed_iters == 0)
        goto done;
    or_precond(p, r, z);
    apply_mask(z, fixed, n);
    memcpy(pp, z, sizeof(double) * n);
    double rz = dot(r, z, n);
    for (;;) {
        or_apply(p, pp, q);
        apply_mask(q, fixed, n);
        double alpha = rz / dot(pp, q, n);
        for (long i = 0; i < n; i++) {
            x[i] += alpha * pp[i];
            r[i] -= alpha * q[i];
        }
        it++;
        rr = dot(r, r, n);
        if (fixed_iters >= 0) {
            if (it >= fixed_iters)
                break;
        } else {
            if (sqrt(rr) <= tol * bref)
                break;
            if (it >= max_iter) {
                status = -1;
                break;
            }
        }
        or_precond(p, r, z);
        apply_mask(z, fixed, n);
        double rz_new = dot(r, z, n);
        double beta = rz_new / rz;
        rz = rz_new;
        for (long i = 0; i < n; i++)
            pp[i] = z[i] + beta * pp[i];
    }
done:
    if (relres)
        *relres = sqrt(rr) / bref;
    free(r);
    free(z);
    free(pp);
    free(q);
    return status < 0 ? -1 : it;
}

/* ------------------------------------------------------------------------- */
/* Dense direct solve (tiny grids only)                                       */
/* ------------------------------------------------------------------------- */

/* LU factorization with partial pivoting of the n x n row-major matrix A
 * (in place); piv receives the row permutation.  Returns 0, or -1 on a zero
 * pivot. */
int or_lu_factor(double *A, int n, int *piv)
{
    for (int c = 0; c < n; c++) {
        int pr = c;
        double best = fabs(A[(long)c * n + c]);
        for (int i = c + 1; i < n; i++) {
            double v = fabs(A[(long)i * n + c]);
            if (v > best) {
                best = v;
                pr = i;
            }
        }
        piv[c] = pr;
        if (best == 0.0)
            return -1;
        if (pr != c)
            for (int j = 0; j < n; j++) {
                double t = A[(long)c * n + j];
                A[(long)c * n + j] = A[(long)pr * n + j];
                A[(long)pr * n + j] = t;
            }
        double inv = 1.0 / A[(long)c * n + c];
        for (int i = c + 1; i < n; i++) {
            double f = A[(long)i * n + c] * inv;
            A[(long)i * n + c] = f;
            if (f != 0.0)
                for (int j = c + 1; j < n; j++)
                    A[(long)i * n + j] -= f * A[(long)c * n + j];
        }
    }
    return 0;
}

void or_lu_solve(const double *LU, int n, const int *piv, double *b)
{
    for (int c = 0; c < n; c++)
        if (piv[c] != c) {
            double t = b[c];
            b[c] = b[piv[c]];
            b[piv[c]] = t;
        }
    for (int i = 0; i < n; i++) {
        double s = b[i];
        for (int j = 0; j < i; j++)
            s -= LU[(long)i * n + j] * b[j];
        b[i] = s;
    }
    for (int i = n - 1; i >= 0; i--) {
        double s = b[i];
        for (int j = i + 1; j < n; j++)
            s -= LU[(long)i * n + j] * b[j];
        b[i] = s / LU[(long)i * n + i];
    }
}

/* Dense matrix of the operator, column c = A e_c (n_dof x n_dof, row major). */
void or_assemble(const or_prob *p, double *Adense)
{
    long n = (long)p->d * nvox(p);
    double *e = calloc(n, sizeof(double));
    double *col = malloc(sizeof(double) * n);
    for (long c = 0; c < n; c++) {
        e[c] = 1.0;
        or_apply(p, e, col);
        e[c] = 0.0;
        for (long r = 0; r < n; r++)
            Adense[r * n + c] = col[r];
    }
    free(col);
    free(e);
}

/* Constrained solve by elimination: x[fixed] are given, A_ff x_f = b_f - A_fc x_c. */
int or_dense_constrained(const or_prob *p, const double *Adense, const double *b,
                         const uint8_t *fixed, double *x)
{
    long n = (long)p->d * nvox(p);
    int nf = 0;
    int *map = malloc(sizeof(int) * n);
    for (long i = 0; i < n; i++)
        map[i] = (fixed && fixed[i]) ? -1 : nf++;
    double *Aff = malloc(sizeof(double) * (long)nf * nf);
    double *rhs = malloc(sizeof(double) * nf);
    int *piv = malloc(sizeof(int) * (nf > 0 ? nf : 1));
    for (long i = 0; i < n; i++) {
        if (map[i] < 0)
            continue;
        double s = b[i];
        for (long j = 0; j < n; j++) {
            if (map[j] < 0)
                s -= Adense[i * n + j] * x[j];
            else
                Aff[(long)map[i] * nf + map[j]] = Adense[i * n + j];
        }
        rhs[map[i]] = s;
    }
    int st = or_lu_factor(Aff, nf, piv);
    if (st == 0) {
        or_lu_solve(Aff, nf, piv, rhs);
        for (long i = 0; i < n; i++)
            if (map[i] >= 0)
                x[i] = rhs[map[i]];
    }
    free(piv);
    free(rhs);
    free(Aff);
    free(map);
    return st;
}

/* ------------------------------------------------------------------------- */
/* Green-matrix route: eqs. (f_discrete), (solve_green), (g), (G)             */
/* ------------------------------------------------------------------------- */

/* Build G (nd x nd, nd = d * n_gamma, row major) from the unit-force solves:
 * column d p + j is the Gamma trace of the solution of A u = e_j delta_p.
 * iters (optional) receives the iteration count of each column solve. */
int or_green_matrix(const or_prob *p, const int64_t *gidx, int n_gamma, double tol, int max_iter,
                    double *G, int *iters)
{
    int d = p->d;
    long N = nvox(p), n = (long)d * N;
    int nd = d * n_gamma;
    double *f = calloc(n, sizeof(double));
    double *u = malloc(sizeof(double) * n);
    for (int pt = 0; pt < n_gamma; pt++)
        for (int j = 0; j < d; j++) {
            f[j * N + gidx[pt]] = 1.0;
            memset(u, 0, sizeof(double) * n);
            int it = or_pcg(p, f, u, NULL, 1.0, tol, max_iter, -1, NULL);
            f[j * N + gidx[pt]] = 0.0;
            if (iters)
                iters[d * pt + j] = it;
            if (it < 0) {
                free(u);
                free(f);
                return -1;
            }
            for (int q = 0; q < n_gamma; q++)
                for (int i = 0; i < d; i++)
                    G[(long)(d * q + i) * nd + (d * pt + j)] = u[i * N + gidx[q]];
        }
    free(u);
    free(f);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Newmark time stepping (eq. Newmark, Algorithm 2)                           */
/* ------------------------------------------------------------------------- */
enum { OR_ROUTE_PROJECTED = 0, OR_ROUTE_GREEN = 1, OR_ROUTE_DENSE = 2 };

typedef struct {
    int route;
    double tol;
    int max_iter;
    double green_tol;
    const int *replay; /* per step: 1 (projected) or 2 (green: u_b, u_f) counts, -1 = use tol */
} or_opts;

/*
 * Run n_steps Newmark steps from (u0, v0) (NULL = 0).  U holds the prescribed
 * displacement, d values per step (uniform on Gamma) when per_point == 0,
 * or d * n_gamma values per step (point major) otherwise.  u_hist receives
 * the displacement after every step (n_steps x d x N), F_hist (optional) the
 * Gamma force (n_steps x d*n_gamma), iters (optional) the iteration counts
 * (n_steps x 2; second entry -1 on the projected route).  v_out and a_out
 * (optional) receive the final velocity and acceleration.
 */
int or_newmark(const or_prob *p, const int64_t *gidx, int n_gamma, const or_opts *o, int n_steps,
               const double *U, int per_point, const double *u0, const double *v0, double *u_hist,
               double *F_hist, int *iters, double *v_out, double *a_out)
{
    int d = p->d;
    long N = nvox(p), n = (long)d * N;
    int nd = d * n_gamma;
    double c = p->beta * p->dt * p->dt, dt = p->dt, gam = p->gamma_nm;
    double *u = calloc(n, sizeof(double)), *v = calloc(n, sizeof(double)),
           *a = calloc(n, sizeof(double)), *ut = malloc(sizeof(double) * n),
           *b = malloc(sizeof(double) * n), *w = malloc(sizeof(double) * n),
           *un = malloc(sizeof(double) * n), *ufp = calloc(n, sizeof(double)),
           *f = calloc(n, sizeof(double));
    uint8_t *fixed = calloc(n, 1);
    double *G = NULL, *Adense = NULL;
    int *piv = NULL;
    int status = 0;
    if (u0)
        memcpy(u, u0, sizeof(double) * n);
    if (v0)
        memcpy(v, v0, sizeof(double) * n);
    for (int pt = 0; pt < n_gamma; pt++)
        for (int j = 0; j < d; j++)
            fixed[j * N + gidx[pt]] = 1;
    /* initial acceleration: a0 = (div(C : grad^s u0) - c v0) / rho */
    or_div_stress(p, u, a);
    for (int j = 0; j < d; j++)
        for (long x = 0; x < N; x++) {
            int g = p->phase[x];
            a[j * N + x] = (a[j * N + x] - (p->damp ? p->damp[g] * v[j * N + x] : 0.0)) / p->rho[g];
        }
    if (o->route == OR_ROUTE_GREEN && n_gamma > 0) {
        G = malloc(sizeof(double) * (long)nd * nd);
        piv = malloc(sizeof(int) * nd);
        if (or_green_matrix(p, gidx, n_gamma, o->green_tol, o->max_iter, G, NULL) != 0 ||
            or_lu_factor(G, nd, piv) != 0) {
            status = -2;
            goto out;
        }
    }
    if (o->route == OR_ROUTE_DENSE) {
        Adense = malloc(sizeof(double) * n * n);
        or_assemble(p, Adense);
    }
    for (int s = 0; s < n_steps; s++) {
        const double *Us = U + (long)s * (per_point ? nd : d);
        /* predictor and right-hand side, eq. (Fourier_ND_b); with viscous damping
         * (rho + gamma dt c) u~ - beta dt^2 c v~, v~ = v + (1 - gamma) dt a */
        for (int j = 0; j < d; j++)
            for (long x = 0; x < N; x++) {
                long i = j * N + x;
                int g = p->phase[x];
                ut[i] = u[i] + dt * v[i] + dt * dt * (0.5 - p->beta) * a[i];
                b[i] = rho_op(p, g) * ut[i];
                if (p->damp)
                    b[i] -= c * p->damp[g] * (v[i] + (1.0 - gam) * dt * a[i]);
            }
        int it1 = -1, it2 = -1, failed = 0;
        int rp1 = o->replay ? o->replay[2 * s] : -1, rp2 = o->replay ? o->replay[2 * s + 1] : -1;
        if (o->route == OR_ROUTE_GREEN && n_gamma > 0) {
            /* u_b: A u_b = b, from u_{n-1} */
            memcpy(un, u, sizeof(double) * n);
            it1 = or_pcg(p, b, un, NULL, sqrt(dot(b, b, n)), o->tol, o->max_iter, rp1, NULL);
            failed |= it1 < 0;
            /* V = U - u_b|Gamma ; F = G^-1 V / (beta dt^2) */
            double *F = malloc(sizeof(double) * nd);
            for (int pt = 0; pt < n_gamma; pt++)
                for (int j = 0; j < d; j++)
                    F[d * pt + j] = (per_point ? Us[d * pt + j] : Us[j]) - un[j * N + gidx[pt]];
            or_lu_solve(G, nd, piv, F);
            for (int t = 0; t < nd; t++)
                F[t] /= c;
            memset(f, 0, sizeof(double) * n);
            for (int pt = 0; pt < n_gamma; pt++)
                for (int j = 0; j < d; j++)
                    f[j * N + gidx[pt]] = F[d * pt + j];
            /* u_f: A u_f = f, from the previous step's u_f */
            it2 = or_pcg(p, f, ufp, NULL, sqrt(dot(f, f, n)), o->tol, o->max_iter, rp2, NULL);
            failed |= it2 < 0;
            for (long i = 0; i < n; i++)
                un[i] += c * ufp[i];
            if (F_hist)
                memcpy(F_hist + (long)s * nd, F, sizeof(double) * nd);
            free(F);
        } else {
            /* constrained solution: A u = b off Gamma, u = U on Gamma */
            memcpy(un, u, sizeof(double) * n);
            for (int pt = 0; pt < n_gamma; pt++)
                for (int j = 0; j < d; j++)
                    un[j * N + gidx[pt]] = per_point ? Us[d * pt + j] : Us[j];
            if (o->route == OR_ROUTE_DENSE) {
                if (or_dense_constrained(p, Adense, b, fixed, un) != 0) {
                    status = -2;
                    goto out;
                }
            } else {
                /* reference norm ||P (b - A ubar)||, ubar = U on Gamma, 0 elsewhere */
                memset(f, 0, sizeof(double) * n);
                for (int pt = 0; pt < n_gamma; pt++)
                    for (int j = 0; j < d; j++)
                        f[j * N + gidx[pt]] = un[j * N + gidx[pt]];
                or_apply(p, f, w);
                for (long i = 0; i < n; i++)
                    w[i] = fixed[i] ? 0.0 : b[i] - w[i];
                double bref = sqrt(dot(w, w, n));
                it1 = or_pcg(p, b, un, fixed, bref, o->tol, o->max_iter, rp1, NULL);
                failed |= it1 < 0;
            }
            if (F_hist) {
                /* reaction on Gamma: (A u - b) / (beta dt^2) */
                or_apply(p, un, w);
                for (int pt = 0; pt < n_gamma; pt++)
                    for (int j = 0; j < d; j++)
                        F_hist[(long)s * nd + d * pt + j] =
                            (w[j * N + gidx[pt]] - b[j * N + gidx[pt]]) / c;
            }
        }
        if (failed) {
            status = -1;
            goto out;
        }
        if (iters) {
            iters[2 * s] = it1;
            iters[2 * s + 1] = it2;
        }
        /* corrector */
        for (long i = 0; i < n; i++) {
            double an = (un[i] - ut[i]) / c;
            v[i] = v[i] + dt * ((1.0 - gam) * a[i] + gam * an);
            a[i] = an;
            u[i] = un[i];
        }
        memcpy(u_hist + (long)s * n, u, sizeof(double) * n);
    }
    if (v_out)
        memcpy(v_out, v, sizeof(double) * n);
    if (a_out)
        memcpy(a_out, a, sizeof(double) * n);
out:
    free(u); free(v); free(a); free(ut); free(b); free(w); free(un); free(ufp); free(f);
    free(fixed); free(G); free(piv); free(Adense);
    return status;
}

/* ------------------------------------------------------------------------- */
/* Explicit central-difference scheme (section 2.3)                           */
/* ------------------------------------------------------------------------- */

/*
 * Newmark with beta = 0, gamma = 1/2 (eq. Central_diff_rule): per step
 *     u_n   = u_{n-1} + dt v_{n-1} + dt^2/2 a_{n-1}
 *     vb    = v_{n-1} + dt/2 a_{n-1} + dt/(2 rho) div(C : grad^s u_n)   (eq. b_explicit, 3D form)
 *     f_n   = 2 rho / dt (Udot_n - vb) on Gamma, 0 elsewhere
 *     v_n   = vb + dt/(2 rho) f_n                      (eq. Explicit_linear_momentum_arranged_3D)
 *     a_n   = (div(C : grad^s u_n) + f_n) / rho        (so that v_n = v_{n-1} + dt/2 (a_{n-1} + a_n))
 * The velocity is prescribed on Gamma (Udot: d values per step, uniform on Gamma, when
 * per_point == 0, else d * n_gamma values per step, point major).  The initial
 * acceleration is a0 = div(C : grad^s u0) / rho.  p->beta and p->gamma_nm are not used.
 * u_hist (n_steps x d x N), v_hist and F_hist (n_steps x d * n_gamma, the nodal force f_n
 * on Gamma) may be NULL; v_out and a_out receive the final velocity and acceleration.
 */
int or_explicit(const or_prob *p, const int64_t *gidx, int n_gamma, int n_steps, const double *Udot,
                int per_point, const double *u0, const double *v0, double *u_hist, double *v_hist,
                double *F_hist, double *v_out, double *a_out)
{
    int d = p->d;
    long N = nvox(p), n = (long)d * N;
    int nd = d * n_gamma;
    double dt = p->dt;
    double *u = calloc(n, sizeof(double)), *v = calloc(n, sizeof(double)),
           *a = calloc(n, sizeof(double)), *sd = malloc(sizeof(double) * n),
           *f = malloc(sizeof(double) * n);
    if (u0)
        memcpy(u, u0, sizeof(double) * n);
    if (v0)
        memcpy(v, v0, sizeof(double) * n);
    or_div_stress(p, u, a);
    for (int j = 0; j < d; j++)
        for (long x = 0; x < N; x++)
            a[j * N + x] /= p->rho[p->phase[x]];
    for (int s = 0; s < n_steps; s++) {
        const double *Us = Udot + (long)s * (per_point ? nd : d);
        for (long i = 0; i < n; i++)
            u[i] = u[i] + dt * v[i] + 0.5 * dt * dt * a[i];
        or_div_stress(p, u, sd);
        /* vb into v; f zero off Gamma */
        for (int j = 0; j < d; j++)
            for (long x = 0; x < N; x++) {
                long i = j * N + x;
                double r = p->rho[p->phase[x]];
                v[i] = v[i] + 0.5 * dt * a[i] + dt / (2.0 * r) * sd[i];
                f[i] = 0.0;
            }
        for (int pt = 0; pt < n_gamma; pt++)
            for (int j = 0; j < d; j++) {
                long i = j * N + gidx[pt];
                double r = p->rho[p->phase[gidx[pt]]];
                double Ud = per_point ? Us[d * pt + j] : Us[j];
                f[i] = 2.0 * r / dt * (Ud - v[i]);
                if (F_hist)
                    F_hist[(long)s * nd + d * pt + j] = f[i];
            }
        for (int j = 0; j < d; j++)
            for (long x = 0; x < N; x++) {
                long i = j * N + x;
                double r = p->rho[p->phase[x]];
                v[i] = v[i] + dt / (2.0 * r) * f[i];
                a[i] = (sd[i] + f[i]) / r;
            }
        if (u_hist)
            memcpy(u_hist + (long)s * n, u, sizeof(double) * n);
        if (v_hist)
            memcpy(v_hist + (long)s * n, v, sizeof(double) * n);
    }
    if (v_out)
        memcpy(v_out, v, sizeof(double) * n);
    if (a_out)
        memcpy(a_out, a, sizeof(double) * n);
    free(u); free(v); free(a); free(sd); free(f);
    return 0;
}

/*
 * Largest eigenvalue omega_max^2 of the discrete problem K x = omega^2 rho x, K = -div(C :
 * grad^s .) (section 2.3.3: the stable increment of eq. Courant_stable is 2 / omega_max), by
 * power iteration on rho^-1 K from the start vector x (d x N, overwritten by the last
 * iterate, normalised in the rho-weighted norm).  Returns the Rayleigh quotient
 * x.K x / x.rho x of the last iterate after `iters` products.
 */
double or_omega2_max(const or_prob *p, double *x, int iters)
{
    int d = p->d;
    long N = nvox(p), n = (long)d * N;
    double *y = malloc(sizeof(double) * n);
    double lam = 0.0;
    for (int it = 0; it <= iters; it++) {
        /* normalise: x.rho x = 1 */
        double m = 0.0;
        for (int j = 0; j < d; j++)
            for (long v = 0; v < N; v++)
                m += p->rho[p->phase[v]] * x[j * N + v] * x[j * N + v];
        double sc = 1.0 / sqrt(m);
        for (long i = 0; i < n; i++)
            x[i] *= sc;
        /* y = K x ; lam = x.K x */
        or_div_stress(p, x, y);
        lam = 0.0;
        for (long i = 0; i < n; i++) {
            y[i] = -y[i];
            lam += x[i] * y[i];
        }
        if (it == iters)
            break;
        /* x <- rho^-1 K x */
        for (int j = 0; j < d; j++)
            for (long v = 0; v < N; v++)
                x[j * N + v] = y[j * N + v] / p->rho[p->phase[v]];
    }
    free(y);
    return lam;
}

/* ------------------------------------------------------------------------- */
/* Direct 3x3x3 periodic convolution (learned warm start)                     */
/* ------------------------------------------------------------------------- */

/* y[co][z][y][x] = bias[co] + sum_ci sum_{a,b,c in 0..2}
 *                 w[co][ci][a][b][c] * x[ci][z+a-1][y+b-1][x+c-1]   (indices mod n) */
void or_conv3d_fwd(const double *x, const double *w, const double *bias, double *y, int cin,
                   int cout, const int *n)
{
    int n1 = n[0], n2 = n[1], n3 = n[2];
    long N = (long)n1 * n2 * n3;
    for (int co = 0; co < cout; co++)
        for (int k = 0; k < n3; k++)
            for (int j = 0; j < n2; j++)
                for (int i = 0; i < n1; i++) {
                    double s = bias ? bias[co] : 0.0;
                    for (int ci = 0; ci < cin; ci++)
                        for (int a = 0; a < 3; a++)
                            for (int bb = 0; bb < 3; bb++)
                                for (int cc = 0; cc < 3; cc++) {
                                    int kk = (k + a - 1 + n3) % n3, jj = (j + bb - 1 + n2) % n2,
                                        ii = (i + cc - 1 + n1) % n1;
                                    s += w[(((long)co * cin + ci) * 3 + a) * 9 + bb * 3 + cc] *
                                         x[ci * N + ((long)kk * n2 + jj) * n1 + ii];
                                }
                    y[co * N + ((long)k * n2 + j) * n1 + i] = s;
                }
}

/* Gradient of L with respect to x, given dL/dy. */
void or_conv3d_bwd_data(const double *dy, const double *w, double *dx, int cin, int cout,
                        const int *n)
{
    int n1 = n[0], n2 = n[1], n3 = n[2];
    long N = (long)n1 * n2 * n3;
    memset(dx, 0, sizeof(double) * cin * N);
    for (int co = 0; co < cout; co++)
        for (int k = 0; k < n3; k++)
            for (int j = 0; j < n2; j++)
                for (int i = 0; i < n1; i++) {
                    double g = dy[co * N + ((long)k * n2 + j) * n1 + i];
                    for (int ci = 0; ci < cin; ci++)
                        for (int a = 0; a < 3; a++)
                            for (int bb = 0; bb < 3; bb++)
                                for (int cc = 0; cc < 3; cc++) {
                                    int kk = (k + a - 1 + n3) % n3, jj = (j + bb - 1 + n2) % n2,
                                        ii = (i + cc - 1 + n1) % n1;
                                    dx[ci * N + ((long)kk * n2 + jj) * n1 + ii] +=
                                        w[(((long)co * cin + ci) * 3 + a) * 9 + bb * 3 + cc] * g;
                                }
                }
}

/* Gradients of L with respect to w and bias, given dL/dy. */
void or_conv3d_bwd_weight(const double *x, const double *dy, double *dw, double *db, int cin,
                          int cout, const int *n)
{
    int n1 = n[0], n2 = n[1], n3 = n[2];
    long N = (long)n1 * n2 * n3;
    memset(dw, 0, sizeof(double) * cout * cin * 27);
    if (db)
        memset(db, 0, sizeof(double) * cout);
    for (int co = 0; co < cout; co++)
        for (int k = 0; k < n3; k++)
            for (int j = 0; j < n2; j++)
                for (int i = 0; i < n1; i++) {
                    double g = dy[co * N + ((long)k * n2 + j) * n1 + i];
                    if (db)
                        db[co] += g;
                    for (int ci = 0; ci < cin; ci++)
                        for (int a = 0; a < 3; a++)
                            for (int bb = 0; bb < 3; bb++)
                                for (int cc = 0; cc < 3; cc++) {
                                    int kk = (k + a - 1 + n3) % n3, jj = (j + bb - 1 + n2) % n2,
                                        ii = (i + cc - 1 + n1) % n1;
                                    dw[(((long)co * cin + ci) * 3 + a) * 9 + bb * 3 + cc] +=
                                        g * x[ci * N + ((long)kk * n2 + jj) * n1 + ii];
                                }
                }
}
