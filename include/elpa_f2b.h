/*
 * Full -> band reduction on MI355X (gfx950): the first stage of the
 * two-stage reduction (Kus et al., "Optimizations of the Eigensolvers in the
 * ELPA Library", Sec. 2: the full Hermitian matrix is reduced to a band of
 * semi-bandwidth nbw by blocked Householder transformations, A <- Q^H A Q).
 *
 * Panel p = 0, nbw, 2 nbw, ... while p + nbw < n: the m = n-p-nbw rows below
 * the band of columns [p, p+nbw) are reduced by k = min(nbw, m) Householder
 * reflectors (LAPACK's larfg convention: v[0] = 1, real beta), and the
 * trailing matrix A[p+nbw:, p+nbw:] is updated from both sides with their
 * compact-WY product.  Reflector c = p+i acts on rows [c+nbw, n).
 *
 * Outputs are written for the next steps on the device:
 *   A: the band matrix in full storage (both triangles, zeros outside the
 *      band), input of elpa_band_to_tridiag (elpa_b2t.h);
 *   V, tau: the reflectors in the layout of elpa_bt2_trafo (elpa_bt2.h):
 *      column c of V holds v_c from row c+nbw down (1 at row c+nbw, zeros
 *      above it in the panel's rows), tau[c] for c = 0 .. n-nbw-1.
 */
#ifndef ELPA_F2B_H
#define ELPA_F2B_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/*
 * A: device, n x n Hermitian matrix in full storage, column major, lda >= n;
 *    overwritten with the band matrix.
 * V: device, n x max(n-nbw, 1) elements, column major, ldv >= n (written in
 *    rows [p+nbw, n) of each panel's columns; other entries untouched).
 * tau: device, max(n-nbw, 1) elements.
 * dtype: ELPA_R64 or ELPA_C64; 1 <= nbw <= 256, n >= 1.  Asynchronous on `stream`; the
 * library allocates a workspace in stream order.  Returns ELPA_OK or
 * ELPA_ERR_ARG / _DTYPE / _ALIGN / _NOMEM / _DEVICE (elpa_hh.h); arguments
 * are checked before anything is enqueued; n <= nbw leaves A as it is.
 */
int elpa_full_to_band(int64_t n, int64_t nbw, void *A, int64_t lda, void *V, int64_t ldv,
                      void *tau, int32_t dtype, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* ELPA_F2B_H */
