/*
 * Symmetric tridiagonal eigenproblem T V^ = V^ Lambda on MI355X (gfx950):
 * the step between the two-stage reduction and the two back-transformations
 * (Kus et al., "Optimizations of the Eigensolvers in the ELPA Library",
 * Sec. 2, the tridiagonal eigenvalue problem; the paper names no solver).
 *
 * Method: divide and conquer (Cuppen's rank-one tearing).  T is split
 * recursively in halves down to 1 x 1 blocks; every merge solves
 * diag(Lambda1, Lambda2) + rho z z^T with deflation of negligible z entries
 * and of close eigenvalue pairs (a Givens rotation), the secular equation
 * 1 + rho sum_j z_j^2 / (d_j - lambda) = 0 per root, z recomputed from the
 * roots (Gu and Eisenstat) so that the eigenvectors are orthogonal to working
 * accuracy, and one product of the children's eigenvectors with the merge's.
 *
 * d: device, n doubles (diagonal).  e: device, n-1 doubles (e[i] couples rows
 *    i and i+1; may be null when n == 1).
 * lam: device, n doubles: all eigenvalues in ascending order.
 * Z: device, n x nev, column major, ldz >= n: the eigenvectors of the nev
 *    smallest eigenvalues, in the element type dtype (ELPA_R64, ELPA_R32, or
 *    ELPA_C64 with zero imaginary parts) so that it can feed elpa_hh_trafo
 *    directly.  0 <= nev <= n.
 *
 * The call allocates its workspace (about 5 n^2 doubles) in stream order and
 * synchronises `stream` after uploading the merge tree (n > 1) and once per
 * level of the tree whose merges exceed 256 rows (the host sizes the
 * products from the deflation counts).
 * Returns ELPA_OK or ELPA_ERR_ARG / _DTYPE / _ALIGN / _NOMEM / _DEVICE
 * (elpa_hh.h); arguments are checked before anything is enqueued.  n = 0 is
 * a no-op.
 */
#ifndef ELPA_TRIDIAG_H
#define ELPA_TRIDIAG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

int elpa_tridiag_eigh(int64_t n, int64_t nev, const double *d, const double *e, double *lam,
                      void *Z, int64_t ldz, int32_t dtype, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* ELPA_TRIDIAG_H */
