/*
 * Band -> tridiagonal reduction (bulge chasing) on MI355X (gfx950).
 *
 * The second step of the two-stage reduction (Kus et al., "Optimizations of
 * the Eigensolvers in the ELPA Library", Sec. 2: the band matrix is reduced
 * further to tridiagonal form).  The paper does not give the algorithm; this
 * library reduces one column per chase step: sweep s = 0 .. n-2 eliminates
 * column s, chase step j = 0 .. J(s)-1 (J(s) = ceil((n-1-s)/nbw)) reduces
 * column c (= s for j = 0, else r - nbw) below row r = s+1+j*nbw with a
 * Householder reflector of length L = min(nbw, n-r), applied two-sided
 * (A <- H^H A H) to the rows and columns [max(r-nbw, 0), min(r+L+nbw, n)).
 * Reflectors follow LAPACK's larfg convention (v[0] = 1, beta = -sign(Re
 * alpha) |x|, real subdiagonal).
 *
 * Outputs are written for the tridiagonal -> band back-transformation of
 * elpa_hh.h, directly in device memory: hh and tau in its slot layout
 * (slot-major in generation order, v[0] = 1 stored, zero padded to nbw),
 * ready for elpa_hh_trafo with the same n and nbw.
 */
#ifndef ELPA_B2T_H
#define ELPA_B2T_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/*
 * A: device, n x n Hermitian band matrix of semi-bandwidth nbw in full
 *    storage (both triangles), column major, leading dimension lda >= n;
 *    overwritten (on return it holds the tridiagonal matrix and zeros).
 * d: device, n doubles, the diagonal; e: device, n-1 doubles, the
 *    subdiagonal (real, also for complex input).
 * hh: device, elpa_hh_num_reflectors(n, nbw) * nbw elements of A's type;
 * tau: device, elpa_hh_num_reflectors(n, nbw) elements.
 * dtype: ELPA_R64 or ELPA_C64 (ELPA_R32 is not provided: single-precision
 *    solves keep the reduction in double precision); 1 <= nbw <= 512.
 * Asynchronous on `stream` (a hipStream_t; NULL = the null stream); about
 * 3 n kernel launches, each a bounded set of independent chase steps (steps
 * that touch disjoint entries), in an order equal to the sequential one.
 * Real bands with nbw <= 64 hold each step's blocks in registers and update only
 * the lower triangle (the symmetric two-sided update of the diagonal block
 * as a rank-2 update), reading only A's lower triangle; the upper triangle
 * is written once at the end.  Complex bands and wider real bands update
 * both triangles step by step.
 * Returns ELPA_OK or ELPA_ERR_ARG / _DTYPE / _ALIGN / _DEVICE (elpa_hh.h);
 * arguments are checked before anything is enqueued; n == 1 writes d only.
 */
int elpa_band_to_tridiag(int64_t n, int64_t nbw, void *A, int64_t lda, double *d, double *e,
                         void *hh, void *tau, int32_t dtype, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* ELPA_B2T_H */
