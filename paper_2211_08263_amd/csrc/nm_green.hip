// Dense factorization and solves of the Green matrix on the device (eqs. (G),
// (L-determination_ND) and the LU factorization of Algorithm 2's preprocessing).
//
// The matrix is stored column major with leading dimension n.  Factorization:
// right-looking blocked LU with partial pivoting (panels of kNb columns):
//   per panel column j: pivot search and row swap inside the panel (one block),
//                       scale of the column below the pivot and rank-1 update of
//                       the rest of the panel (one thread per row);
//   row swaps of the panel applied to the columns outside it (one thread per column);
//   U12 = L11^-1 A12 (forward substitution, one thread per column);
//   A22 -= L21 U12 (tiled FP64 GEMM, 64 x 64 tiles staged through LDS).
// Solves: the pivots composed into one permutation (a gather), then blocked forward (unit L)
// and backward (U) substitution in panels of kSb rows, one launch per panel: every block forms
// the panel's solution from the inverted kSb x kSb diagonal block (inverted once after the
// factorization) and updates its share of the remaining rows.
#include "nm_common.h"
#include "nm_green.h"

namespace nm {

constexpr int kNb = 64;    // panel width of the factorization
constexpr int kSb = 256;   // panel width of the substitutions (inverted diagonal blocks)
constexpr int kGT = 64;    // GEMM tile (rows and columns of C per block)

// Pivot search in column j (rows j..n-1) and swap of rows j and p inside the panel
// columns [k0, k1).  One block of 1024 threads.
__global__ __launch_bounds__(1024) void k_lu_pivot(double* __restrict__ A, int n, int j, int k0, int k1,
                                                   int* __restrict__ piv, int* __restrict__ sing)
{
    __shared__ double bv[1024];
    __shared__ int bi[1024];
    const double* col = A + (long)j * n;
    double best = -1.0;
    int bidx = j;
    for (int i = j + threadIdx.x; i < n; i += blockDim.x) {
        const double v = fabs(col[i]);
        if (v > best) {
            best = v;
            bidx = i;
        }
    }
    bv[threadIdx.x] = best;
    bi[threadIdx.x] = bidx;
    __syncthreads();
    // fixed-order tree; ties go to the smaller row index (as a sequential scan would)
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const double o = bv[threadIdx.x + s];
            const int oi = bi[threadIdx.x + s];
            if (o > bv[threadIdx.x] || (o == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
                bv[threadIdx.x] = o;
                bi[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    const int p = bi[0];
    if (threadIdx.x == 0) {
        piv[j] = p;
        if (!(bv[0] > 0.0)) *sing = 1;
    }
    if (p != j) {
        for (int c = k0 + threadIdx.x; c < k1; c += blockDim.x) {
            double* cc = A + (long)c * n;
            const double t = cc[j];
            cc[j] = cc[p];
            cc[p] = t;
        }
    }
}

// Column j below the pivot: l = a / a_jj; then the rest of the panel's rows: a_ic -= l_i a_jc.
__global__ __launch_bounds__(256) void k_lu_update(double* __restrict__ A, int n, int j, int k1)
{
    const int i = j + 1 + blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double* cj = A + (long)j * n;
    const double l = cj[i] / cj[j];
    cj[i] = l;
    for (int c = j + 1; c < k1; c++) {
        double* cc = A + (long)c * n;
        cc[i] -= l * cc[j];
    }
}

// The swaps of rows k0..k1-1 (in order) applied to every column outside [k0, k1).
__global__ __launch_bounds__(256) void k_lu_swaps(double* __restrict__ A, int n, int k0, int k1,
                                                  const int* __restrict__ piv)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n - (k1 - k0)) return;
    if (c >= k0) c += k1 - k0;
    double* cc = A + (long)c * n;
    for (int j = k0; j < k1; j++) {
        const int p = piv[j];
        if (p != j) {
            const double t = cc[j];
            cc[j] = cc[p];
            cc[p] = t;
        }
    }
}

// U12 = L11^-1 A12 for the columns [k1, n): forward substitution with the unit lower
// triangle of rows/columns [k0, k1), one thread per column.
__global__ __launch_bounds__(256) void k_lu_trsm(double* __restrict__ A, int n, int k0, int k1)
{
    const int c = k1 + blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    double* cc = A + (long)c * n;
    for (int r = k0 + 1; r < k1; r++) {
        double s = cc[r];
        for (int q = k0; q < r; q++) s -= A[(long)q * n + r] * cc[q];
        cc[r] = s;
    }
}

// C[m x m'] -= Lp[m x kb] * Up[kb x m'] on the trailing block: rows and columns [k1, n),
// Lp = A[k1:n, k0:k1], Up = A[k0:k1, k1:n] (column major, leading dimension n).  Each
// block computes a 64 x 64 tile of C, each thread a 4 x 4 sub-tile.
__global__ __launch_bounds__(256) void k_lu_gemm(double* __restrict__ A, int n, int k0, int k1)
{
    __shared__ double Ls[kNb][kGT + 1]; // Ls[q][r]: row r of the tile, panel column q
    __shared__ double Us[kNb][kGT + 1]; // Us[q][c]: panel row q, column c of the tile
    const int kb = k1 - k0;
    const int r0 = k1 + blockIdx.y * kGT, c0 = k1 + blockIdx.x * kGT;
    const int tid = threadIdx.x;
    for (int e = tid; e < kb * kGT; e += blockDim.x) {
        // L21 tile: consecutive threads read consecutive rows of one panel column
        const int q = e / kGT, r = e % kGT;
        const int gr = r0 + r;
        Ls[q][r] = gr < n ? A[(long)(k0 + q) * n + gr] : 0.0;
        // U12 tile: consecutive threads read consecutive panel rows of one column
        const int c = e / kb, qq = e % kb;
        const int gc = c0 + c;
        Us[qq][c] = gc < n ? A[(long)gc * n + (k0 + qq)] : 0.0;
    }
    __syncthreads();
    const int tr = (tid % 16) * 4, tc = (tid / 16) * 4;
    double acc[4][4] = {};
    for (int q = 0; q < kb; q++) {
        double a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; i++) {
            a[i] = Ls[q][tr + i];
            b[i] = Us[q][tc + i];
        }
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int jj = 0; jj < 4; jj++) acc[i][jj] += a[i] * b[jj];
    }
#pragma unroll
    for (int jj = 0; jj < 4; jj++) {
        const int gc = c0 + tc + jj;
        if (gc >= n) continue;
        double* cc = A + (long)gc * n;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int gr = r0 + tr + i;
            if (gr < n) cc[gr] -= acc[i][jj];
        }
    }
}

int lu_factor_device(double* A, int n, int* piv, int* sing, hipStream_t s)
{
    for (int k0 = 0; k0 < n; k0 += kNb) {
        const int k1 = k0 + kNb < n ? k0 + kNb : n;
        for (int j = k0; j < k1; j++) {
            hipLaunchKernelGGL(k_lu_pivot, dim3(1), dim3(1024), 0, s, A, n, j, k0, k1, piv, sing);
            const int rows = n - j - 1;
            if (rows > 0)
                hipLaunchKernelGGL(k_lu_update, dim3((rows + 255) / 256), dim3(256), 0, s, A, n, j, k1);
        }
        const int others = n - (k1 - k0);
        if (others > 0) hipLaunchKernelGGL(k_lu_swaps, dim3((others + 255) / 256), dim3(256), 0, s, A, n, k0, k1, piv);
        const int rest = n - k1;
        if (rest > 0) {
            hipLaunchKernelGGL(k_lu_trsm, dim3((rest + 255) / 256), dim3(256), 0, s, A, n, k0, k1);
            const int tiles = (rest + kGT - 1) / kGT;
            hipLaunchKernelGGL(k_lu_gemm, dim3(tiles, tiles), dim3(256), 0, s, A, n, k0, k1);
        }
        if (hipGetLastError() != hipSuccess) return -2;
    }
    return 0;
}

// The row swaps of the factorization composed into one permutation (one thread, once per
// factorization): after the swaps, row i of b holds the original row perm[i].
__global__ void k_lu_perm_from_piv(const int* __restrict__ piv, int* __restrict__ perm, int n)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    for (int i = 0; i < n; i++) perm[i] = i;
    for (int j = 0; j < n; j++) {
        const int p = piv[j];
        if (p != j) {
            const int t = perm[j];
            perm[j] = perm[p];
            perm[p] = t;
        }
    }
}

// Inverses of the kSb x kSb diagonal blocks of the factors (block per diagonal block, kSb
// threads; thread j forms column j): dinv[0 .. kSb^2) = L_kk^-1 (unit lower),
// dinv[kSb^2 .. 2 kSb^2) = U_kk^-1, column major (entry (i, j) at j kSb + i), zero outside the
// triangle.  The rows of the factors are swept in order, each staged once in LDS for all
// columns.
__global__ __launch_bounds__(kSb) void k_lu_diag_inv(const double* __restrict__ A, int n, double* __restrict__ dinv)
{
    __shared__ double row[kSb];
    const int k0 = blockIdx.x * kSb;
    const int kb = n - k0 < kSb ? n - k0 : kSb;
    const int j = threadIdx.x;
    double* Lj = dinv + (long)blockIdx.x * 2 * kSb * kSb + (long)j * kSb; // column j of L_kk^-1
    double* Uj = Lj + kSb * kSb;                                           // column j of U_kk^-1
    for (int i = 0; i < kSb; i++) {
        Lj[i] = 0.0;
        Uj[i] = 0.0;
    }
    // L x = e_j: x_j = 1, x_i = -sum_{j <= q < i} L_iq x_q for i > j (row i of L staged)
    if (j < kb) Lj[j] = 1.0;
    for (int i = 1; i < kb; i++) {
        __syncthreads();
        if (j < i) row[j] = A[(long)(k0 + j) * n + (k0 + i)];
        __syncthreads();
        if (j < i) {
            double acc = 0.0;
            for (int q = j; q < i; q++) acc += row[q] * Lj[q];
            Lj[i] = -acc;
        }
    }
    // U x = e_j: x_j = 1 / U_jj, x_i = -(sum_{i < q <= j} U_iq x_q) / U_ii for i < j (row i of U
    // staged, rows from the bottom)
    if (j < kb) Uj[j] = 1.0 / A[(long)(k0 + j) * n + (k0 + j)];
    for (int i = kb - 2; i >= 0; i--) {
        __syncthreads();
        if (j >= i && j < kb) row[j] = A[(long)(k0 + j) * n + (k0 + i)];
        __syncthreads();
        if (j > i && j < kb) {
            double acc = 0.0;
            for (int q = i + 1; q <= j; q++) acc += row[q] * Uj[q];
            Uj[i] = -acc / row[i];
        }
    }
}

int lu_prepare_solve(const double* LU, int n, const int* piv, int* perm, double* dinv, hipStream_t s)
{
    hipLaunchKernelGGL(k_lu_perm_from_piv, dim3(1), dim3(1), 0, s, piv, perm, n);
    const int np = (n + kSb - 1) / kSb;
    hipLaunchKernelGGL(k_lu_diag_inv, dim3(np), dim3(kSb), 0, s, LU, n, dinv);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

__global__ __launch_bounds__(256) void k_lu_gather(const double* __restrict__ b, const int* __restrict__ perm,
                                                   double* __restrict__ w, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) w[i] = b[perm[i]];
}

// One panel of a substitution: x_k = D_k in[k0:k1] with D_k the inverted diagonal block
// (every block forms it; block 0 stores it in out[k0:k1]), then in[r] -= A[r, k0:k1] x_k for
// the rows r in [r0, r1) (one thread per row).  Those rows lie outside [k0, k1), so no block
// reads an entry another block writes.
__global__ __launch_bounds__(kSb) void k_tri_panel(const double* __restrict__ A, int n, const double* __restrict__ D,
                                                   double* __restrict__ in, double* __restrict__ out, int k0, int k1,
                                                   int r0, int r1)
{
    __shared__ double xs[kSb];
    __shared__ double bk[kSb];
    const int t = threadIdx.x;
    const int kb = k1 - k0;
    bk[t] = t < kb ? in[k0 + t] : 0.0;
    __syncthreads();
    {
        double acc = 0.0;
        if (t < kb)
            for (int q = 0; q < kb; q++) acc += D[q * kSb + t] * bk[q];
        xs[t] = acc;
    }
    __syncthreads();
    if (blockIdx.x == 0 && t < kb) out[k0 + t] = xs[t];
    const int r = r0 + blockIdx.x * blockDim.x + t;
    if (r < r1) {
        double acc = 0.0;
        for (int q = 0; q < kb; q++) acc += A[(long)(k0 + q) * n + r] * xs[q];
        in[r] -= acc;
    }
}

int lu_solve_device(const double* LU, int n, const int* perm, const double* dinv, double* b, double* work,
                    hipStream_t s)
{
    double* w = work;      // P b, then the forward residuals
    double* y = work + n;  // L^-1 P b, then the backward residuals
    hipLaunchKernelGGL(k_lu_gather, dim3((n + 255) / 256), dim3(256), 0, s, b, perm, w, n);
    const int np = (n + kSb - 1) / kSb;
    for (int k = 0; k < np; k++) {
        const int k0 = k * kSb, k1 = k0 + kSb < n ? k0 + kSb : n;
        const int rows = n - k1;
        hipLaunchKernelGGL(k_tri_panel, dim3(rows > 0 ? (rows + kSb - 1) / kSb : 1), dim3(kSb), 0, s, LU, n,
                           dinv + (long)k * 2 * kSb * kSb, w, y, k0, k1, k1, n);
    }
    for (int k = np - 1; k >= 0; k--) {
        const int k0 = k * kSb, k1 = k0 + kSb < n ? k0 + kSb : n;
        hipLaunchKernelGGL(k_tri_panel, dim3(k0 > 0 ? (k0 + kSb - 1) / kSb : 1), dim3(kSb), 0, s, LU, n,
                           dinv + (long)k * 2 * kSb * kSb + kSb * kSb, y, b, k0, k1, 0, k0);
    }
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

// Column dst of G (column major) from the gathered Gamma trace: G[d q + i][dst] = g[3 q + i].
__global__ __launch_bounds__(256) void k_green_column(double* __restrict__ G, long nd, long dst,
                                                      const double* __restrict__ g, long ng, int d)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ng * d) return;
    const long q = e / d;
    const int i = (int)(e % d);
    G[dst * nd + d * q + i] = g[3 * q + i];
}

int launch_green_column(double* G, long nd, long dst, const double* g, long ng, int d, hipStream_t s)
{
    const long n = ng * d;
    hipLaunchKernelGGL(k_green_column, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, G, nd, dst, g, ng, d);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

// V (dim*ng, point major) = U - u_b|Gamma from the gathered trace gb (3 per point) and the
// prescribed values U (3 per point when per_point, else 3 values).
__global__ __launch_bounds__(256) void k_green_rhs(double* __restrict__ V, const double* __restrict__ gb,
                                                   const double* __restrict__ U, int per_point, long ng, int d)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ng * d) return;
    const long p = e / d;
    const int j = (int)(e % d);
    V[e] = (per_point ? U[3 * p + j] : U[j]) - gb[3 * p + j];
}

int launch_green_rhs(double* V, const double* gb, const double* U, int per_point, long ng, int d, hipStream_t s)
{
    const long n = ng * d;
    if (n == 0) return 0;
    hipLaunchKernelGGL(k_green_rhs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, V, gb, U, per_point, ng, d);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

// F3 (3 per point) = F (dim per point) * scale, third component zero in 2D.
__global__ __launch_bounds__(256) void k_green_force(double* __restrict__ F3, double* __restrict__ F,
                                                     double scale, long ng, int d)
{
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= ng) return;
    for (int j = 0; j < 3; j++) {
        double v = 0.0;
        if (j < d) {
            v = F[d * p + j] * scale;
            F[d * p + j] = v;
        }
        F3[3 * p + j] = v;
    }
}

int launch_green_force(double* F3, double* F, double scale, long ng, int d, hipStream_t s)
{
    if (ng == 0) return 0;
    hipLaunchKernelGGL(k_green_force, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, s, F3, F, scale, ng, d);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

} // namespace nm
