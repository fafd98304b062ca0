// Device-side dense kernels of the Green-matrix route (implemented in nm_green.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nm {

// LU factorization with partial pivoting of the n x n column-major matrix A in place
// (unit lower L below the diagonal, U on and above it); piv[j] is the row swapped with
// row j at step j.  *sing (device) is set to 1 when a pivot is zero.  Asynchronous.
int lu_factor_device(double* A, int n, int* piv, int* sing, hipStream_t s);
// After lu_factor_device: the pivots composed into one row permutation (perm, n ints) and the
// inverses of the 256 x 256 diagonal blocks (dinv, 2 * 256 * 256 doubles per 256 columns), so
// that a solve is one gather and one launch per panel and direction.  Asynchronous.
int lu_prepare_solve(const double* LU, int n, const int* piv, int* perm, double* dinv, hipStream_t s);
// b <- A^-1 b with those factors; work: 2 n doubles.  Asynchronous.
int lu_solve_device(const double* LU, int n, const int* perm, const double* dinv, double* b, double* work,
                    hipStream_t s);
// Column dst of the column-major G (leading dimension nd) from a Gamma trace g (3 values
// per point): G[d q + i][dst] = g[3 q + i].
int launch_green_column(double* G, long nd, long dst, const double* g, long ng, int d, hipStream_t s);
// V[d p + j] = U_p,j - gb[3 p + j] (U: 3 values per point when per_point, else 3 values).
int launch_green_rhs(double* V, const double* gb, const double* U, int per_point, long ng, int d, hipStream_t s);
// F <- scale F in place (d per point) and F3 = the same with 3 components per point.
int launch_green_force(double* F3, double* F, double scale, long ng, int d, hipStream_t s);

} // namespace nm
