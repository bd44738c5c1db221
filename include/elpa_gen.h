/*
 * Generalized Hermitian-definite eigenproblem A V = B V Lambda on MI355X
 * (gfx950): the steps around the standard solve (Kus et al., "Optimizations
 * of the Eigensolvers in the ELPA Library", Sec. 2, Eq. (1), the Cholesky
 * factorisation B = L L^H, the forward transformation A~ = L^{-1} A L^{-H} and
 * the back-transformation V = L^{-H} V~; Sec. 4, "Generalized EVP problem":
 * the factor is inverted once and the inverse is kept in B's storage, so
 * later problems with the same B skip the factorisation).
 *
 * All matrices are device memory, column major, fp64 (ELPA_R64) or complex
 * fp64 (ELPA_C64).  Calls are asynchronous on `stream` (a hipStream_t, 0 for
 * the default stream); a workspace, where one is needed, is allocated in
 * stream order and freed before the call returns.  Every call checks its
 * arguments before enqueueing anything and returns ELPA_OK or ELPA_ERR_ARG /
 * _DTYPE / _ALIGN / _NOMEM / _DEVICE (elpa_hh.h).  n = 0 is a no-op.
 */
#ifndef ELPA_GEN_H
#define ELPA_GEN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/*
 * B <- L^{-1}, where B = L L^H (the Cholesky factorisation) and L is lower
 * triangular with a positive real diagonal.
 *
 * B: n x n, ldb >= n; only its lower triangle is read.  On return the lower
 *    triangle holds L^{-1}, the strict upper triangle zeros.
 * info: device int32, written in stream order: 0, or j + 1 (1-based, LAPACK's
 *    convention) when the leading minor of order j + 1 is not positive
 *    definite (B's contents are then unspecified).  The caller reads it after
 *    synchronising the stream.
 * n and ldb must be below 2^31.
 */
int elpa_cholesky_inverse(int64_t n, void *B, int64_t ldb, int32_t dtype, void *stream,
                          int32_t *info);

/*
 * A <- Linv A Linv^H, made exactly Hermitian (A[j][i] = conj(A[i][j]), real
 * diagonal).  A: n x n Hermitian in full storage (both triangles read),
 * lda >= n.  Linv: n x n lower triangular (the output of
 * elpa_cholesky_inverse; its strict upper triangle is not read), ldl >= n.
 */
int elpa_generalized_to_standard(int64_t n, void *A, int64_t lda, const void *Linv, int64_t ldl,
                                 int32_t dtype, void *stream);

/*
 * Q <- Linv^H Q: eigenvectors of the standard problem to those of the
 * generalized one.  Q: n x nev, ldq >= n.  Linv as above.
 */
int elpa_generalized_back(int64_t n, int64_t nev, const void *Linv, int64_t ldl, void *Q,
                          int64_t ldq, int32_t dtype, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* ELPA_GEN_H */
