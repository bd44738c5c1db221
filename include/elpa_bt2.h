/*
 * Band -> full back-transformation of eigenvectors on MI355X (gfx950).
 *
 * The two-stage solver (Kus et al., "Optimizations of the Eigensolvers in the
 * ELPA Library", Sec. 2) first reduces the full matrix to a band of
 * semi-bandwidth nbw with blocked Householder transformations; after the band
 * eigenvectors are known (tridiagonal solve, then the tridiagonal -> band
 * back-transformation of elpa_hh.h), they are multiplied by the orthogonal /
 * unitary matrix of that first stage.  This header declares that second
 * back-transformation.
 *
 * Reflectors: c = 0 .. n-nbw-1 (none when n <= nbw), in the order the first
 * stage generated them (column c of the matrix, panel by panel).  Reflector c
 * is H_c = I - tau[c] v_c v_c^H with v_c supported on rows [c+nbw, n):
 *   v_c[0] = 1 at row c+nbw (the value stored there is not read),
 *   v_c[i] = V[(c+nbw+i) + c*ldv] for i = 1 .. n-c-nbw-1.
 * Entries of column c on or above row c+nbw are never read (so V may be the
 * lower part of the reduced matrix itself, as LAPACK keeps its vectors).
 *
 * Operation, in place on Q (n x nev, column major, leading dimension ldq):
 *     Q <- H_0 H_1 ... H_{n-nbw-1} Q.
 *
 * Element types and error codes are those of elpa_hh.h (ELPA_R64, ELPA_R32,
 * ELPA_C64; ELPA_OK, ELPA_ERR_*).  Pointers are device pointers aligned to
 * the element size; tau holds max(0, n-nbw) elements.  Calls are
 * asynchronous on `stream` (a hipStream_t; NULL = the null stream); the
 * library allocates its workspace in stream order and frees it the same way.
 * Rows ldq > n of Q are not touched.  Invalid arguments are reported before
 * anything is enqueued.
 */
#ifndef ELPA_BT2_H
#define ELPA_BT2_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/*
 * The operation above, in blocks of `block` consecutive reflectors applied as
 * compact-WY products I - V T V^H (0 = library choice, otherwise 1 .. 512).
 * Errors: ELPA_ERR_ARG (negative sizes, nbw < 1, ldq < n, ldv < n, a NULL
 * pointer where work is to be done, block out of range), ELPA_ERR_DTYPE,
 * ELPA_ERR_ALIGN, ELPA_ERR_NOMEM, ELPA_ERR_DEVICE.
 */
int elpa_bt2_trafo(int64_t n, int64_t nev, int64_t nbw, const void *V, int64_t ldv,
                   const void *tau, void *Q, int64_t ldq, int32_t dtype, void *stream,
                   int64_t block);

/*
 * Device workspace (bytes) elpa_bt2_trafo allocates for these sizes and block
 * (0 = library choice); -1 for invalid arguments.
 */
int64_t elpa_bt2_workspace_bytes(int64_t n, int64_t nev, int64_t nbw, int32_t dtype,
                                 int64_t block);

#ifdef __cplusplus
}
#endif

#endif /* ELPA_BT2_H */
