/*
 * Plain CPU oracle for the two-stage Hermitian eigensolver.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code with the HIP library.
 *
 * Everything here is written for obviousness, not speed: fp64 throughout,
 * compiled without FMA contraction (-ffp-contract=off -fno-fast-math), loops in
 * the order the mathematics states them, OpenMP only over independent columns
 * (back-transformation) or independent eigenvalues / clusters (tridiagonal
 * solver).
 *
 * Paper: Kus et al., "Optimizations of the Eigensolvers in the ELPA Library",
 * Sec. 2 (the eigenvalue problem solved by ELPA): the Householder matrices
 * Q_i = I - beta_i v_i v_i^H are never formed, only their vectors are kept
 * (Eq. tridiagonalization and the text after it); the two-stage method reduces
 * full -> band -> tridiagonal and back-transforms every eigenvector twice.
 *
 * Indexing (0-based) of the band -> tridiagonal reflectors, b = nbw:
 *   sweep s = 0 .. n-2, chase step j = 0 .. J(s)-1, J(s) = ceil((n-1-s)/b),
 *   row start r = s+1+j*b, length L = min(b, n-r).
 *   Slots are numbered in generation order (s ascending, then j ascending);
 *   slot k owns hh[k*b .. k*b+b-1] with v[0] = 1 stored and zero padding
 *   past L, and tau[k].  H(s,j) = I - tau v v^H.
 */
#include <complex.h>
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double _Complex zdbl;

/* ------------------------------------------------------------------ */
/* slot arithmetic                                                      */
/* ------------------------------------------------------------------ */

int64_t orc_num_steps(int64_t n, int64_t b, int64_t s)
{
    if (s < 0 || s > n - 2) return 0;
    return (n - 1 - s + b - 1) / b;
}

/* Total number of reflector slots: a plain sum over the sweeps. */
int64_t orc_num_reflectors(int64_t n, int64_t b)
{
    int64_t tot = 0;
    for (int64_t s = 0; s <= n - 2; ++s) tot += orc_num_steps(n, b, s);
    return tot;
}

/* ------------------------------------------------------------------ */
/* Householder generation (LAPACK larfg convention, no safmin scaling): */
/* on return x[0] = 1, x[1:] = v[1:], and H^H x_in = beta e_0 with beta */
/* real, where H = I - tau v v^H.                                        */
/* ------------------------------------------------------------------ */

void orc_larfg_d(int64_t L, double *x, double *tau, double *beta)
{
    double alpha = x[0], ss = 0.0;
    for (int64_t i = 1; i < L; ++i) ss += x[i] * x[i];
    double xnorm = sqrt(ss);
    if (xnorm == 0.0) {
        *tau = 0.0;
        *beta = alpha;
        x[0] = 1.0;
        return;
    }
    double h = sqrt(alpha * alpha + ss);
    double bt = (alpha >= 0.0) ? -h : h;
    *tau = (bt - alpha) / bt;
    double sc = 1.0 / (alpha - bt);
    for (int64_t i = 1; i < L; ++i) x[i] *= sc;
    x[0] = 1.0;
    *beta = bt;
}

void orc_larfg_z(int64_t L, zdbl *x, zdbl *tau, double *beta)
{
    zdbl alpha = x[0];
    double ar = creal(alpha), ai = cimag(alpha), ss = 0.0;
    for (int64_t i = 1; i < L; ++i) ss += creal(x[i] * conj(x[i]));
    if (ss == 0.0 && ai == 0.0) {
        *tau = 0.0;
        *beta = ar;
        x[0] = 1.0;
        return;
    }
    double h = sqrt(ar * ar + ai * ai + ss);
    double bt = (ar >= 0.0) ? -h : h;
    *tau = (bt - ar) / bt + I * (-ai / bt);
    zdbl sc = 1.0 / (alpha - bt);
    for (int64_t i = 1; i < L; ++i) x[i] *= sc;
    x[0] = 1.0;
    *beta = bt;
}

/* ------------------------------------------------------------------ */
/* Stage 2: band -> tridiagonal by one-column-per-step bulge chasing.   */
/* A is a full n x n Hermitian matrix (both triangles stored, column    */
/* major, leading dimension lda) with semi-bandwidth b; it is           */
/* overwritten.  For every slot (s, j) in generation order the column   */
/* c (= s for j = 0, else r - b) is reduced below row r by a reflector  */
/* on rows [r, r+L), applied two-sided as A <- H^H A H.  Nonzeros of    */
/* rows/columns [r, r+L) never reach beyond b outside that range, so    */
/* the update is restricted to the window [r-b, r+L+b).                  */
/* Outputs: d (n), e (n-1), hh (nrefl*b), tau (nrefl).                  */
/* ------------------------------------------------------------------ */

#define AD(i, k) A[(i) + (int64_t)(k) * lda]

int orc_band_to_tridiag_d(int64_t n, int64_t b, double *A, int64_t lda,
                          double *d, double *e, double *hh, double *tau)
{
    if (n < 1 || b < 1 || lda < n) return -1;
    double *v = (double *)malloc(sizeof(double) * (size_t)b);
    if (!v) return -2;
    int64_t slot = 0;
    for (int64_t s = 0; s <= n - 2; ++s) {
        int64_t J = orc_num_steps(n, b, s);
        for (int64_t j = 0; j < J; ++j, ++slot) {
            int64_t r = s + 1 + j * b;
            int64_t L = (b < n - r) ? b : n - r;
            int64_t c = (j == 0) ? s : r - b;
            for (int64_t i = 0; i < L; ++i) v[i] = AD(r + i, c);
            double t, beta;
            orc_larfg_d(L, v, &t, &beta);
            int64_t lo = (r - b > 0) ? r - b : 0;
            int64_t hi = (r + L + b < n) ? r + L + b : n;
            if (t != 0.0) {
                /* left: rows [r, r+L) of columns [lo, hi) <- H^H * rows */
                for (int64_t k = lo; k < hi; ++k) {
                    double w = 0.0;
                    for (int64_t i = 0; i < L; ++i) w += v[i] * AD(r + i, k);
                    w *= t;
                    for (int64_t i = 0; i < L; ++i) AD(r + i, k) -= v[i] * w;
                }
                /* right: columns [r, r+L) of rows [lo, hi) <- cols * H */
                for (int64_t i = lo; i < hi; ++i) {
                    double w = 0.0;
                    for (int64_t q = 0; q < L; ++q) w += AD(i, r + q) * v[q];
                    w *= t;
                    for (int64_t q = 0; q < L; ++q) AD(i, r + q) -= w * v[q];
                }
            }
            AD(r, c) = beta;
            AD(c, r) = beta;
            for (int64_t i = 1; i < L; ++i) {
                AD(r + i, c) = 0.0;
                AD(c, r + i) = 0.0;
            }
            double *dst = hh + slot * b;
            for (int64_t i = 0; i < b; ++i) dst[i] = (i < L) ? v[i] : 0.0;
            tau[slot] = t;
        }
    }
    for (int64_t i = 0; i < n; ++i) d[i] = AD(i, i);
    for (int64_t i = 0; i + 1 < n; ++i) e[i] = AD(i + 1, i);
    free(v);
    return 0;
}

int orc_band_to_tridiag_z(int64_t n, int64_t b, zdbl *A, int64_t lda,
                          double *d, double *e, zdbl *hh, zdbl *tau)
{
    if (n < 1 || b < 1 || lda < n) return -1;
    zdbl *v = (zdbl *)malloc(sizeof(zdbl) * (size_t)b);
    if (!v) return -2;
    int64_t slot = 0;
    for (int64_t s = 0; s <= n - 2; ++s) {
        int64_t J = orc_num_steps(n, b, s);
        for (int64_t j = 0; j < J; ++j, ++slot) {
            int64_t r = s + 1 + j * b;
            int64_t L = (b < n - r) ? b : n - r;
            int64_t c = (j == 0) ? s : r - b;
            for (int64_t i = 0; i < L; ++i) v[i] = AD(r + i, c);
            zdbl t;
            double beta;
            orc_larfg_z(L, v, &t, &beta);
            int64_t lo = (r - b > 0) ? r - b : 0;
            int64_t hi = (r + L + b < n) ? r + L + b : n;
            if (t != 0.0) {
                /* left: H^H = I - conj(tau) v v^H */
                for (int64_t k = lo; k < hi; ++k) {
                    zdbl w = 0.0;
                    for (int64_t i = 0; i < L; ++i) w += conj(v[i]) * AD(r + i, k);
                    w *= conj(t);
                    for (int64_t i = 0; i < L; ++i) AD(r + i, k) -= v[i] * w;
                }
                /* right: H = I - tau v v^H */
                for (int64_t i = lo; i < hi; ++i) {
                    zdbl w = 0.0;
                    for (int64_t q = 0; q < L; ++q) w += AD(i, r + q) * v[q];
                    w *= t;
                    for (int64_t q = 0; q < L; ++q) AD(i, r + q) -= w * conj(v[q]);
                }
            }
            AD(r, c) = beta;
            AD(c, r) = beta;
            for (int64_t i = 1; i < L; ++i) {
                AD(r + i, c) = 0.0;
                AD(c, r + i) = 0.0;
            }
            zdbl *dst = hh + slot * b;
            for (int64_t i = 0; i < b; ++i) dst[i] = (i < L) ? v[i] : 0.0;
            tau[slot] = t;
        }
    }
    for (int64_t i = 0; i < n; ++i) d[i] = creal(AD(i, i));
    for (int64_t i = 0; i + 1 < n; ++i) e[i] = creal(AD(i + 1, i));
    free(v);
    return 0;
}

#undef AD

/* ------------------------------------------------------------------ */
/* Back-transformation tridiagonal -> band (the hot path's definition): */
/*   Q <- H(0,0) H(0,1) ... H(n-2, J-1) Q                                */
/* i.e. the last generated reflector is applied first: s descending,    */
/* and j descending inside a sweep.  Q is n x nev, column major, ldq.   */
/* Columns are independent; threads take blocks of 8 columns.           */
/* ------------------------------------------------------------------ */

static int64_t *slot_offsets(int64_t n, int64_t b)
{
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 1 ? n : 1));
    if (!off) return NULL;
    int64_t acc = 0;
    for (int64_t s = 0; s <= n - 2; ++s) {
        off[s] = acc;
        acc += orc_num_steps(n, b, s);
    }
    return off;
}

#define ORC_CB 8

int orc_bt1_d(int64_t n, int64_t nev, int64_t b, const double *hh,
              const double *tau, double *Q, int64_t ldq, int nthreads)
{
    if (n <= 1 || nev <= 0) return 0;
    if (b < 1 || ldq < n) return -1;
    int64_t *off = slot_offsets(n, b);
    if (!off) return -2;
    int64_t nblk = (nev + ORC_CB - 1) / ORC_CB;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
    for (int64_t blk = 0; blk < nblk; ++blk) {
        int64_t c0 = blk * ORC_CB;
        int64_t c1 = (c0 + ORC_CB < nev) ? c0 + ORC_CB : nev;
        for (int64_t s = n - 2; s >= 0; --s) {
            int64_t J = orc_num_steps(n, b, s);
            for (int64_t j = J - 1; j >= 0; --j) {
                int64_t slot = off[s] + j;
                double t = tau[slot];
                if (t == 0.0) continue;
                const double *v = hh + slot * b;
                int64_t r = s + 1 + j * b;
                int64_t L = (b < n - r) ? b : n - r;
                for (int64_t c = c0; c < c1; ++c) {
                    double *x = Q + r + c * ldq;
                    double w = 0.0;
                    for (int64_t i = 0; i < L; ++i) w += v[i] * x[i];
                    w *= t;
                    for (int64_t i = 0; i < L; ++i) x[i] -= v[i] * w;
                }
            }
        }
    }
    free(off);
    return 0;
}

int orc_bt1_z(int64_t n, int64_t nev, int64_t b, const zdbl *hh,
              const zdbl *tau, zdbl *Q, int64_t ldq, int nthreads)
{
    if (n <= 1 || nev <= 0) return 0;
    if (b < 1 || ldq < n) return -1;
    int64_t *off = slot_offsets(n, b);
    if (!off) return -2;
    int64_t nblk = (nev + ORC_CB - 1) / ORC_CB;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
    for (int64_t blk = 0; blk < nblk; ++blk) {
        int64_t c0 = blk * ORC_CB;
        int64_t c1 = (c0 + ORC_CB < nev) ? c0 + ORC_CB : nev;
        for (int64_t s = n - 2; s >= 0; --s) {
            int64_t J = orc_num_steps(n, b, s);
            for (int64_t j = J - 1; j >= 0; --j) {
                int64_t slot = off[s] + j;
                zdbl t = tau[slot];
                if (t == 0.0) continue;
                const zdbl *v = hh + slot * b;
                int64_t r = s + 1 + j * b;
                int64_t L = (b < n - r) ? b : n - r;
                for (int64_t c = c0; c < c1; ++c) {
                    zdbl *x = Q + r + c * ldq;
                    zdbl w = 0.0;
                    for (int64_t i = 0; i < L; ++i) w += conj(v[i]) * x[i];
                    w *= t;
                    for (int64_t i = 0; i < L; ++i) x[i] -= v[i] * w;
                }
            }
        }
    }
    free(off);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Tridiagonal eigensolver: Sturm-sequence bisection for the wanted     */
/* eigenvalues, then inverse iteration with modified Gram-Schmidt       */
/* inside clusters.  T has diagonal d (n) and off-diagonal e (n-1).     */
/* ------------------------------------------------------------------ */

/* number of eigenvalues of T smaller than x (LDL^T inertia) */
int64_t orc_sturm_count(int64_t n, const double *d, const double *e, double x,
                        double pivmin)
{
    int64_t cnt = 0;
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) ++cnt;
    for (int64_t i = 1; i < n; ++i) {
        q = d[i] - x - (e[i - 1] * e[i - 1]) / q;
        if (fabs(q) < pivmin) q = -pivmin;
        if (q < 0.0) ++cnt;
    }
    return cnt;
}

static double tri_pivmin(int64_t n, const double *e)
{
    double m = 1.0;
    for (int64_t i = 0; i + 1 < n; ++i)
        if (e[i] * e[i] > m) m = e[i] * e[i];
    return DBL_MIN * m;
}

static double tri_norm1(int64_t n, const double *d, const double *e)
{
    double nrm = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double s = fabs(d[i]);
        if (i > 0) s += fabs(e[i - 1]);
        if (i + 1 < n) s += fabs(e[i]);
        if (s > nrm) nrm = s;
    }
    return nrm;
}

/* eigenvalues il..iu (0-based, ascending, inclusive) by bisection */
int orc_tridiag_bisect(int64_t n, const double *d, const double *e, int64_t il,
                       int64_t iu, double *w, int nthreads)
{
    if (n < 1 || il < 0 || iu >= n || il > iu) return -1;
    const double eps = DBL_EPSILON;
    double pivmin = tri_pivmin(n, e);
    double gl = d[0], gu = d[0];
    for (int64_t i = 0; i < n; ++i) {
        double rad = 0.0;
        if (i > 0) rad += fabs(e[i - 1]);
        if (i + 1 < n) rad += fabs(e[i]);
        if (d[i] - rad < gl) gl = d[i] - rad;
        if (d[i] + rad > gu) gu = d[i] + rad;
    }
    double tnorm = fmax(fabs(gl), fabs(gu));
    gl -= 2.0 * eps * tnorm * (double)n + 4.0 * pivmin;
    gu += 2.0 * eps * tnorm * (double)n + 4.0 * pivmin;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
#endif
    for (int64_t k = il; k <= iu; ++k) {
        double lo = gl, hi = gu;
        for (int it = 0; it < 200; ++it) {
            double tol = 2.0 * eps * fmax(fabs(lo), fabs(hi)) + pivmin;
            if (hi - lo <= tol) break;
            double mid = 0.5 * (lo + hi);
            if (orc_sturm_count(n, d, e, mid, pivmin) > k)
                hi = mid;
            else
                lo = mid;
        }
        w[k - il] = 0.5 * (lo + hi);
    }
    return 0;
}

/* deterministic uniform(-1,1) stream (splitmix64) for start vectors */
static uint64_t sm64(uint64_t *st)
{
    uint64_t z = (*st += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static double unif_pm1(uint64_t *st)
{
    return 2.0 * ((double)(sm64(st) >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
}

/* LU with partial pivoting of T - lam*I (row interchanges), then solve */
typedef struct {
    double *u0, *u1, *u2, *mult;
    char *swp;
} tri_lu;

static void tri_factor(int64_t n, const double *d, const double *e, double lam,
                       double tiny, tri_lu *f)
{
    double p0 = d[0] - lam, p1 = (n > 1) ? e[0] : 0.0, p2 = 0.0;
    for (int64_t i = 0; i + 1 < n; ++i) {
        double nx0 = e[i], nx1 = d[i + 1] - lam, nx2 = (i + 2 < n) ? e[i + 1] : 0.0;
        if (fabs(p0) >= fabs(nx0)) {
            if (fabs(p0) < tiny) p0 = (p0 < 0.0) ? -tiny : tiny;
            double m = nx0 / p0;
            f->u0[i] = p0; f->u1[i] = p1; f->u2[i] = p2;
            f->mult[i] = m; f->swp[i] = 0;
            p0 = nx1 - m * p1;
            p1 = nx2 - m * p2;
            p2 = 0.0;
        } else {
            double m = p0 / nx0;
            f->u0[i] = nx0; f->u1[i] = nx1; f->u2[i] = nx2;
            f->mult[i] = m; f->swp[i] = 1;
            double q0 = p1 - m * nx1, q1 = p2 - m * nx2;
            p0 = q0; p1 = q1; p2 = 0.0;
        }
    }
    if (fabs(p0) < tiny) p0 = (p0 < 0.0) ? -tiny : tiny;
    f->u0[n - 1] = p0; f->u1[n - 1] = 0.0; f->u2[n - 1] = 0.0;
}

static void tri_solve(int64_t n, const tri_lu *f, double *x)
{
    for (int64_t i = 0; i + 1 < n; ++i) {
        if (f->swp[i]) {
            double t = x[i];
            x[i] = x[i + 1];
            x[i + 1] = t - f->mult[i] * x[i];
        } else {
            x[i + 1] -= f->mult[i] * x[i];
        }
    }
    for (int64_t i = n - 1; i >= 0; --i) {
        double s = x[i];
        if (i + 1 < n) s -= f->u1[i] * x[i + 1];
        if (i + 2 < n) s -= f->u2[i] * x[i + 2];
        x[i] = s / f->u0[i];
    }
}

static double nrm2(int64_t n, const double *x)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += x[i] * x[i];
    return sqrt(s);
}

/*
 * Eigenvectors for the ascending eigenvalues w[0..m-1] (m = iu-il+1, as
 * returned by orc_tridiag_bisect).  Z is n x m, column major, ldz >= n.
 * Consecutive eigenvalues closer than ||T||_1 / n form a cluster; vectors in
 * a cluster are orthogonalised against the earlier ones of the cluster by
 * modified Gram-Schmidt after every solve.  Sign: largest-magnitude entry > 0.
 */
int orc_tridiag_invit(int64_t n, const double *d, const double *e, int64_t m,
                      const double *w, double *Z, int64_t ldz, uint64_t seed,
                      int nthreads)
{
    if (n < 1 || m < 0 || m > n || ldz < n) return -1;
    if (m == 0) return 0;
    const double eps = DBL_EPSILON;
    double tn = tri_norm1(n, d, e);
    double tiny = eps * (tn > 0.0 ? tn : 1.0);
    double gap_cl = (tn > 0.0 ? tn : 1.0) / (double)n;
    /* cluster boundaries */
    int64_t *cstart = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m + 1));
    if (!cstart) return -2;
    int64_t nc = 0;
    cstart[nc++] = 0;
    for (int64_t k = 1; k < m; ++k)
        if (w[k] - w[k - 1] >= gap_cl) cstart[nc++] = k;
    cstart[nc] = m;
    int err = 0;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads) reduction(| : err)
#endif
    for (int64_t ci = 0; ci < nc; ++ci) {
        tri_lu f;
        f.u0 = (double *)malloc(sizeof(double) * (size_t)n);
        f.u1 = (double *)malloc(sizeof(double) * (size_t)n);
        f.u2 = (double *)malloc(sizeof(double) * (size_t)n);
        f.mult = (double *)malloc(sizeof(double) * (size_t)n);
        f.swp = (char *)malloc((size_t)n);
        if (!f.u0 || !f.u1 || !f.u2 || !f.mult || !f.swp) {
            err |= 1;
        } else {
            double prev_shift = -INFINITY;
            for (int64_t k = cstart[ci]; k < cstart[ci + 1]; ++k) {
                double lam = w[k];
                double pert = 10.0 * eps * fmax(fabs(lam), tiny);
                if (lam - prev_shift < pert) lam = prev_shift + pert;
                prev_shift = lam;
                tri_factor(n, d, e, lam, tiny, &f);
                double *z = Z + k * ldz;
                uint64_t st = seed ^ (0x5851F42D4C957F2DULL * (uint64_t)(k + 1));
                for (int64_t i = 0; i < n; ++i) z[i] = unif_pm1(&st);
                double s0 = nrm2(n, z);
                for (int64_t i = 0; i < n; ++i) z[i] /= s0;
                double growth_need = 1.0 / (10.0 * sqrt((double)n) * eps * (tn > 0 ? tn : 1.0));
                for (int it = 0; it < 5; ++it) {
                    tri_solve(n, &f, z);
                    for (int64_t p = cstart[ci]; p < k; ++p) {
                        const double *zp = Z + p * ldz;
                        double dot = 0.0;
                        for (int64_t i = 0; i < n; ++i) dot += zp[i] * z[i];
                        for (int64_t i = 0; i < n; ++i) z[i] -= dot * zp[i];
                    }
                    double nz = nrm2(n, z);
                    for (int64_t i = 0; i < n; ++i) z[i] /= nz;
                    if (it >= 2 && nz >= growth_need) break;
                }
                /* sign: the entry of largest magnitude is positive */
                int64_t imax = 0;
                for (int64_t i = 1; i < n; ++i)
                    if (fabs(z[i]) > fabs(z[imax])) imax = i;
                if (z[imax] < 0.0)
                    for (int64_t i = 0; i < n; ++i) z[i] = -z[i];
            }
        }
        free(f.u0); free(f.u1); free(f.u2); free(f.mult); free(f.swp);
    }
    free(cstart);
    return err ? -2 : 0;
}
