// Divide and conquer for the symmetric tridiagonal eigenproblem (C ABI in
// include/elpa_tridiag.h; Kus et al., Sec. 2).
//
// Tearing: every boundary b between rows b and b+1 is the split point of one
// node of the halving tree, so T = blockdiag(T1', T2') + rho v v^T with
// rho = |e_b|, v = [e_last; sign(e_b) e_first], and the diagonal entries
// next to every boundary are lowered by |e_b| once, before the leaves.
//
// A merge of node [lo, hi) (split at mid, s rows) with the children's sorted
// eigenvalues in L[lo, mid) and L[mid, hi) and eigenvectors in the diagonal
// blocks of Q:
//   prep:     z = [last row of Q1; sign(e) first row of Q2] / sqrt(2),
//             rho' = 2 rho; the two sorted lists merged by rank; deflation
//             scan in sorted order (tol = 8 eps max(|D|, |z|)): rho'|z_p| <=
//             tol deflates p; else if the previous candidate pj is close,
//             |(D_p - D_pj) c s| <= tol with c = z_p/r, s = -z_pj/r,
//             r = hypot(z_p, z_pj), the pair is rotated so that z_pj = 0 and
//             pj deflates; the K survivors (delta, w) are strictly increasing;
//   gather:   W = the block's columns in sorted order, zeros outside each
//             column's child; rotate: the recorded rotations applied to W;
//   secular:  root i in (delta_i, delta_i+1) (the last one in (delta_K-1,
//             delta_K-1 + rho' |w|^2]) as delta_o + tau, o the nearer pole,
//             by Newton's method kept inside a shrinking bracket (one wave
//             per root, the sums over the poles split over its lanes);
//   zhat:     w^_j^2 = (lambda_K-1 - delta_j)/rho' prod_{i<j} (lambda_i -
//             delta_j)/(delta_i - delta_j) prod_{j<=i<K-1} (lambda_i -
//             delta_j)/(delta_i+1 - delta_j), sign of w_j;
//   vec:      U[:, i] = w^ / (delta - lambda_i), normalised;
//   product:  Out = W[:, survivors] U; above 256 rows as two products on the
//             halves, the survivors grouped by the rows they can be nonzero
//             in (child 1 only, both after a rotation, child 2 only);
//   final:    every value's rank among the merge's s values; L and Q's block
//             rewritten in ascending order.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <mutex>
#include <vector>

#include "../../include/elpa_hh.h"
#include "../../include/elpa_tridiag.h"
#include "wy_blas.h"

namespace edc {

struct Node {
  int64_t lo, mid, hi, woff;
};

constexpr int kSmall = 256;  // merges up to this size use the in-kernel product
constexpr double kEps = 1.1102230246251565e-16;  // 2^-53

struct Ws {
  double *Q, *L, *Ds, *zs, *delta, *wv, *rc, *rs, *tau, *zh, *vals;
  int32_t *perm, *ndl, *dfl, *ra, *rb, *org, *rflag, *gidx;
  int32_t *K, *ndf, *nrot, *grp;
  double* rho;
  double *Wg, *Qc, *U, *Out;
};

__global__ __launch_bounds__(256) void k_init(int64_t n, const double* __restrict__ d,
                                              const double* __restrict__ e, double* __restrict__ L,
                                              double* __restrict__ Q) {
  const int64_t tot = n * n;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < tot;
       x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = x % n, j = x / n;
    Q[x] = i == j ? 1.0 : 0.0;
    if (j == 0) L[i] = d[i] - (i > 0 ? fabs(e[i - 1]) : 0.0) - (i + 1 < n ? fabs(e[i]) : 0.0);
  }
}

__device__ __forceinline__ double block_max(double v, double* red) {
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double r = red[0];
  for (int k = 1; k < (int)(blockDim.x >> 6); ++k) r = fmax(r, red[k]);
  return r;
}

__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double r = red[0];
  for (int k = 1; k < (int)(blockDim.x >> 6); ++k) r += red[k];
  return r;
}

// One workgroup (256 threads) per merge.
__global__ __launch_bounds__(256) void k_prep(const Node* __restrict__ nodes, int64_t n,
                                              const double* __restrict__ e, Ws w) {
  __shared__ double red[4];
  const Node nd = nodes[blockIdx.x];
  const int64_t lo = nd.lo, mid = nd.mid, s = nd.hi - nd.lo, s1 = nd.mid - nd.lo;
  const double beta = e[mid - 1];
  const double th = beta >= 0.0 ? 1.0 : -1.0;
  const double rho2 = 2.0 * fabs(beta);
  const double r2 = 0.70710678118654752440;  // 1/sqrt(2)
  double dmax = 0.0, zmax = 0.0;
  for (int64_t t = threadIdx.x; t < s; t += blockDim.x) {
    double val, zv;
    int64_t rank;
    if (t < s1) {
      val = w.L[lo + t];
      zv = w.Q[(lo + t) * n + (mid - 1)] * r2;
      int64_t a = 0, b = s - s1;  // number of child-2 values < val
      while (a < b) {
        const int64_t c = (a + b) >> 1;
        if (w.L[mid + c] < val) a = c + 1; else b = c;
      }
      rank = t + a;
    } else {
      const int64_t j = t - s1;
      val = w.L[mid + j];
      zv = th * w.Q[(mid + j) * n + mid] * r2;
      int64_t a = 0, b = s1;  // number of child-1 values <= val
      while (a < b) {
        const int64_t c = (a + b) >> 1;
        if (w.L[lo + c] <= val) a = c + 1; else b = c;
      }
      rank = j + a;
    }
    w.perm[lo + rank] = (int32_t)t;
    w.Ds[lo + rank] = val;
    w.zs[lo + rank] = zv;
    w.rflag[lo + t] = 0;
    dmax = fmax(dmax, fabs(val));
    zmax = fmax(zmax, fabs(zv));
  }
  dmax = block_max(dmax, red);
  zmax = block_max(zmax, red);
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double tol = 8.0 * kEps * fmax(dmax, zmax);
  double* Ds = w.Ds + lo;
  double* zs = w.zs + lo;
  int32_t K = 0, ndf = 0, nrot = 0;
  int64_t pj = -1;
  double dpj = 0.0, zpj = 0.0;  // the candidate's current values
  for (int64_t p = 0; p < s; ++p) {
    double dp = Ds[p], zp = zs[p];
    if (rho2 * fabs(zp) <= tol) {
      w.dfl[lo + ndf++] = (int32_t)p;
      continue;
    }
    if (pj < 0) {
      pj = p, dpj = dp, zpj = zp;
      continue;
    }
    const double r = hypot(zp, zpj);
    const double c = zp / r, sn = -zpj / r;
    const double t = dp - dpj;
    if (fabs(t * c * sn) <= tol) {
      const double t2 = dpj * c * c + dp * sn * sn;
      dp = dpj * sn * sn + dp * c * c;
      zp = r;
      Ds[pj] = t2;
      zs[pj] = 0.0;
      Ds[p] = dp;
      zs[p] = zp;
      w.ra[lo + nrot] = (int32_t)pj;
      w.rb[lo + nrot] = (int32_t)p;
      w.rc[lo + nrot] = c;
      w.rs[lo + nrot] = sn;
      ++nrot;
      w.rflag[lo + pj] = 1;
      w.rflag[lo + p] = 1;
      w.dfl[lo + ndf++] = (int32_t)pj;
    } else {
      w.ndl[lo + K] = (int32_t)pj;
      w.delta[lo + K] = dpj;
      w.wv[lo + K] = zpj;
      ++K;
    }
    pj = p, dpj = dp, zpj = zp;
  }
  if (pj >= 0) {
    w.ndl[lo + K] = (int32_t)pj;
    w.delta[lo + K] = dpj;
    w.wv[lo + K] = zpj;
    ++K;
  }
  // survivors grouped by the rows their column can be nonzero in: child 1
  // only, both (rotated), child 2 only; gidx = the column of Qc (and row of U)
  int32_t g[3] = {0, 0, 0};
  for (int32_t j = 0; j < K; ++j) {
    const int32_t pos = w.ndl[lo + j];
    ++g[w.rflag[lo + pos] ? 1 : (w.perm[lo + pos] < s1 ? 0 : 2)];
  }
  int32_t c[3] = {0, g[0], g[0] + g[1]};
  for (int32_t j = 0; j < K; ++j) {
    const int32_t pos = w.ndl[lo + j];
    w.gidx[lo + j] = c[w.rflag[lo + pos] ? 1 : (w.perm[lo + pos] < s1 ? 0 : 2)]++;
  }
  w.grp[3 * blockIdx.x] = g[0];
  w.grp[3 * blockIdx.x + 1] = g[1];
  w.grp[3 * blockIdx.x + 2] = g[2];
  w.K[blockIdx.x] = K;
  w.ndf[blockIdx.x] = ndf;
  w.nrot[blockIdx.x] = nrot;
  w.rho[blockIdx.x] = rho2;
}

// Flattened grid: block b -> merge b / per, item (b % per) * 256 + tid.
__device__ __forceinline__ void split_idx(int64_t per, int64_t& m, int64_t& base) {
  m = (int64_t)blockIdx.x / per;
  base = ((int64_t)blockIdx.x % per) * blockDim.x;
}

// W[:, p] = column perm[p] of the block, zeros outside its child's rows.
// One workgroup per (merge, column).
__global__ __launch_bounds__(256) void k_gather(const Node* __restrict__ nodes, int64_t n,
                                                int64_t smax, Ws w) {
  const int64_t m = (int64_t)blockIdx.x / smax, p = (int64_t)blockIdx.x % smax;
  const Node nd = nodes[m];
  const int64_t lo = nd.lo, s = nd.hi - nd.lo, s1 = nd.mid - nd.lo;
  if (p >= s) return;
  const int64_t t = w.perm[lo + p];
  const int64_t r0 = t < s1 ? 0 : s1, r1 = t < s1 ? s1 : s;
  const double* __restrict__ src = w.Q + (lo + t) * n + lo;
  double* __restrict__ dst = w.Wg + nd.woff + p * s;
  for (int64_t r = threadIdx.x; r < s; r += blockDim.x)
    dst[r] = (r >= r0 && r < r1) ? src[r] : 0.0;
}

// The rotations in recorded order, one thread per row.
__global__ __launch_bounds__(256) void k_rotate(const Node* __restrict__ nodes, int64_t per,
                                                Ws w) {
  int64_t m, base;
  split_idx(per, m, base);
  const Node nd = nodes[m];
  const int64_t lo = nd.lo, s = nd.hi - nd.lo, r = base + threadIdx.x;
  const int32_t nrot = w.nrot[m];
  if (r >= s || nrot == 0) return;
  double* __restrict__ W = w.Wg + nd.woff;
  for (int32_t q = 0; q < nrot; ++q) {
    const int64_t a = w.ra[lo + q], b = w.rb[lo + q];
    const double c = w.rc[lo + q], sn = w.rs[lo + q];
    const double x = W[a * s + r], y = W[b * s + r];
    W[a * s + r] = c * x + sn * y;
    W[b * s + r] = c * y - sn * x;
  }
}

__device__ __forceinline__ double wave_sum(double v) {
  // butterfly: every lane ends with the same bits (a + b == b + a)
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Root i of 1 + rho sum_j w_j^2 / (delta_j - lambda) = 0, one wave per root:
// the lanes split the sums over j and every lane takes the same decisions.
__global__ __launch_bounds__(256) void k_secular(const Node* __restrict__ nodes, int64_t per,
                                                 Ws w) {
  const int64_t m = (int64_t)blockIdx.x / per;
  const int lane = threadIdx.x & 63;
  const int64_t i = ((int64_t)blockIdx.x % per) * 4 + (threadIdx.x >> 6);
  const Node nd = nodes[m];
  const int64_t lo = nd.lo;
  const int64_t K = w.K[m];
  if (i >= K) return;
  const double rho = w.rho[m];
  const double* __restrict__ dl = w.delta + lo;
  const double* __restrict__ wv = w.wv + lo;
  int64_t o;
  double tlo, thi;
  if (i < K - 1) {
    const double a = dl[i], h = 0.5 * (dl[i + 1] - a);
    double g = 0.0;
    for (int64_t j = lane; j < K; j += 64) g += wv[j] * wv[j] / ((dl[j] - a) - h);
    g = 1.0 + rho * wave_sum(g);
    if (g >= 0.0) o = i, tlo = 0.0, thi = h;
    else o = i + 1, tlo = -h, thi = 0.0;
  } else {
    double sw = 0.0;
    for (int64_t j = lane; j < K; j += 64) sw += wv[j] * wv[j];
    o = i, tlo = 0.0, thi = rho * wave_sum(sw);
  }
  const double sg = dl[o];
  double t = 0.5 * (tlo + thi);
  for (int it = 0; it < 200; ++it) {
    double g = 0.0, gp = 0.0, ab = 0.0;
    for (int64_t j = lane; j < K; j += 64) {
      const double D = (dl[j] - sg) - t;
      const double term = wv[j] * wv[j] / D;
      g += term;
      gp += term / D;
      ab += fabs(term);
    }
    g = 1.0 + rho * wave_sum(g);
    gp = rho * wave_sum(gp);
    ab = wave_sum(ab);
    if (fabs(g) <= kEps * (double)(K + 1) * (1.0 + rho * ab)) break;
    if (g < 0.0) tlo = t; else thi = t;
    double tn = t - g / gp;
    if (!(tn > tlo && tn < thi)) tn = 0.5 * (tlo + thi);
    if (thi - tlo <= 2.0 * kEps * fmax(fabs(tlo), fabs(thi))) break;
    t = tn;
  }
  if (lane == 0) {
    w.org[lo + i] = (int32_t)o;
    w.tau[lo + i] = t;
  }
}

__global__ __launch_bounds__(256) void k_zhat(const Node* __restrict__ nodes, int64_t per, Ws w) {
  int64_t m, base;
  split_idx(per, m, base);
  const Node nd = nodes[m];
  const int64_t lo = nd.lo, j = base + threadIdx.x;
  const int64_t K = w.K[m];
  if (j >= K) return;
  const double rho = w.rho[m];
  const double* __restrict__ dl = w.delta + lo;
  const int32_t* __restrict__ org = w.org + lo;
  const double* __restrict__ tau = w.tau + lo;
  const double dj = dl[j];
  double pr = ((dl[org[K - 1]] - dj) + tau[K - 1]) / rho;
  for (int64_t i = 0; i < j; ++i) pr *= ((dl[org[i]] - dj) + tau[i]) / (dl[i] - dj);
  for (int64_t i = j; i < K - 1; ++i) pr *= ((dl[org[i]] - dj) + tau[i]) / (dl[i + 1] - dj);
  w.zh[lo + j] = copysign(sqrt(fmax(pr, 0.0)), w.wv[lo + j]);
}

// U[gidx[j], i] (ld s) = zhat_j / (delta_j - lambda_i), normalised; one
// workgroup per (merge, column).
__global__ __launch_bounds__(256) void k_vec(const Node* __restrict__ nodes, int64_t smax, Ws w) {
  __shared__ double red[4];
  const int64_t m = (int64_t)blockIdx.x / smax, i = (int64_t)blockIdx.x % smax;
  const Node nd = nodes[m];
  const int64_t lo = nd.lo, s = nd.hi - nd.lo;
  const int64_t K = w.K[m];
  if (i >= K) return;
  const double* __restrict__ dl = w.delta + lo;
  const double sg = dl[w.org[lo + i]], t = w.tau[lo + i];
  double ss = 0.0;
  for (int64_t j = threadIdx.x; j < K; j += blockDim.x) {
    const double u = w.zh[lo + j] / ((dl[j] - sg) - t);
    ss += u * u;
  }
  const double nrm = sqrt(block_sum(ss, red));
  double* __restrict__ U = w.U + nd.woff + i * s;
  for (int64_t j = threadIdx.x; j < K; j += blockDim.x)
    U[w.gidx[lo + j]] = (w.zh[lo + j] / ((dl[j] - sg) - t)) / nrm;
}

// Qc[:, gidx[j]] (ld s) = W[:, survivor j]; one workgroup per (merge, column).
__global__ __launch_bounds__(256) void k_compress(const Node* __restrict__ nodes, int64_t smax,
                                                  Ws w) {
  const int64_t m = (int64_t)blockIdx.x / smax, j = (int64_t)blockIdx.x % smax;
  const Node nd = nodes[m];
  const int64_t lo = nd.lo, s = nd.hi - nd.lo;
  if (j >= w.K[m]) return;
  const double* __restrict__ src = w.Wg + nd.woff + (int64_t)w.ndl[lo + j] * s;
  double* __restrict__ dst = w.Qc + nd.woff + (int64_t)w.gidx[lo + j] * s;
  for (int64_t r = threadIdx.x; r < s; r += blockDim.x) dst[r] = src[r];
}

// C[0:rows, 0:cols] = 0 (ld ldc).
__global__ __launch_bounds__(256) void k_zero(double* __restrict__ C, int64_t ldc, int64_t rows,
                                              int64_t cols) {
  const int64_t tot = rows * cols;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < tot;
       x += (int64_t)gridDim.x * blockDim.x)
    C[(x / rows) * ldc + x % rows] = 0.0;
}

// Out = Qc U for merges of at most 256 rows: one workgroup per merge, a
// thread per row.
__global__ __launch_bounds__(256) void k_gemm_small(const Node* __restrict__ nodes, Ws w) {
  const Node nd = nodes[blockIdx.x];
  const int64_t s = nd.hi - nd.lo, r = threadIdx.x;
  const int64_t K = w.K[blockIdx.x];
  if (r >= s) return;
  const double* __restrict__ Qc = w.Qc + nd.woff;
  const double* __restrict__ U = w.U + nd.woff;
  double* __restrict__ Out = w.Out + nd.woff;
  for (int64_t i = 0; i < K; ++i) {
    double acc = 0.0;
    for (int64_t j = 0; j < K; ++j) acc = fma(Qc[j * s + r], U[i * s + j], acc);
    Out[i * s + r] = acc;
  }
}

// vals[lo + x]: x < K the roots, then the deflated values.
__global__ __launch_bounds__(256) void k_vals(const Node* __restrict__ nodes, int64_t per, Ws w) {
  int64_t m, base;
  split_idx(per, m, base);
  const Node nd = nodes[m];
  const int64_t lo = nd.lo, s = nd.hi - nd.lo, x = base + threadIdx.x;
  if (x >= s) return;
  const int64_t K = w.K[m];
  w.vals[lo + x] = x < K ? w.delta[lo + w.org[lo + x]] + w.tau[lo + x]
                         : w.Ds[lo + w.dfl[lo + (x - K)]];
}

// Rank of value x among the merge's s values (ties by index), then L and the
// block of Q rewritten in ascending order.  One workgroup per (merge, x).
__global__ __launch_bounds__(256) void k_final(const Node* __restrict__ nodes, int64_t n,
                                               int64_t smax, Ws w) {
  __shared__ double red[4];
  const int64_t m = (int64_t)blockIdx.x / smax, x = (int64_t)blockIdx.x % smax;
  const Node nd = nodes[m];
  const int64_t lo = nd.lo, s = nd.hi - nd.lo;
  if (x >= s) return;
  const int64_t K = w.K[m];
  const double* __restrict__ v = w.vals + lo;
  const double vx = v[x];
  double cnt = 0.0;
  for (int64_t y = threadIdx.x; y < s; y += blockDim.x)
    cnt += (v[y] < vx || (v[y] == vx && y < x)) ? 1.0 : 0.0;
  const int64_t rank = (int64_t)block_sum(cnt, red);
  const double* __restrict__ src =
      x < K ? w.Out + nd.woff + x * s : w.Wg + nd.woff + (int64_t)w.dfl[lo + (x - K)] * s;
  double* __restrict__ dst = w.Q + (lo + rank) * n + lo;
  for (int64_t r = threadIdx.x; r < s; r += blockDim.x) dst[r] = src[r];
  if (threadIdx.x == 0) w.L[lo + rank] = vx;
}

template <typename E>
__device__ __forceinline__ E cvt(double x);
template <>
__device__ __forceinline__ double cvt<double>(double x) { return x; }
template <>
__device__ __forceinline__ float cvt<float>(double x) { return (float)x; }
template <>
__device__ __forceinline__ ebt::zc cvt<ebt::zc>(double x) { return ebt::zc{x, 0.0}; }

template <typename E>
__global__ __launch_bounds__(256) void k_output(int64_t n, int64_t nev, const double* __restrict__ Q,
                                                E* __restrict__ Z, int64_t ldz) {
  const int64_t tot = n * nev;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < tot;
       x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = x % n, j = x / n;
    Z[j * ldz + i] = cvt<E>(Q[j * n + i]);
  }
}

__global__ __launch_bounds__(256) void k_lam(int64_t n, const double* __restrict__ L,
                                             double* __restrict__ lam) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    lam[i] = L[i];
}

void build_tree(int64_t lo, int64_t hi, int depth, std::vector<std::vector<Node>>& lv) {
  if (hi - lo <= 1) return;
  const int64_t mid = lo + (hi - lo) / 2;
  if ((int)lv.size() <= depth) lv.resize(depth + 1);
  lv[depth].push_back(Node{lo, mid, hi, 0});
  build_tree(lo, mid, depth + 1, lv);
  build_tree(mid, hi, depth + 1, lv);
}

unsigned grid_for(int64_t items) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((items + 255) / 256, 1 << 20));
}

template <typename E>
int run(int64_t n, int64_t nev, const double* d, const double* e, double* lam, E* Z, int64_t ldz,
        hipStream_t st) {
  std::vector<std::vector<Node>> lv;
  build_tree(0, n, 0, lv);
  int64_t wmax = 1, mmax = 1;
  std::vector<int64_t> first(lv.size() + 1, 0);
  for (size_t l = 0; l < lv.size(); ++l) {
    int64_t off = 0;
    for (Node& x : lv[l]) {
      x.woff = off;
      off += (x.hi - x.lo) * (x.hi - x.lo);
    }
    wmax = std::max(wmax, off);
    mmax = std::max<int64_t>(mmax, (int64_t)lv[l].size());
    first[l + 1] = first[l] + (int64_t)lv[l].size();
  }
  std::vector<Node> flat;
  for (auto& l : lv) flat.insert(flat.end(), l.begin(), l.end());

  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  const size_t nd8 = al((size_t)n * 8), ni4 = al((size_t)n * 4), nm8 = al((size_t)mmax * 8),
               nm4 = al((size_t)mmax * 4), big = al((size_t)wmax * 8),
               nodes_b = al(std::max<size_t>(flat.size(), 1) * sizeof(Node));
  const size_t total = al((size_t)n * n * 8) + 10 * nd8 + 8 * ni4 + 3 * nm4 + al((size_t)mmax * 12) + nm8 +
                       4 * big + nodes_b;
  char* ws = nullptr;
  if (hipMallocAsync((void**)&ws, total, st) != hipSuccess) return ELPA_ERR_NOMEM;
  char* p = ws;
  auto take = [&p](size_t b) {
    char* r = p;
    p += b;
    return r;
  };
  Ws w;
  w.Q = (double*)take(al((size_t)n * n * 8));
  w.L = (double*)take(nd8);
  w.Ds = (double*)take(nd8);
  w.zs = (double*)take(nd8);
  w.delta = (double*)take(nd8);
  w.wv = (double*)take(nd8);
  w.rc = (double*)take(nd8);
  w.rs = (double*)take(nd8);
  w.tau = (double*)take(nd8);
  w.zh = (double*)take(nd8);
  w.vals = (double*)take(nd8);
  w.perm = (int32_t*)take(ni4);
  w.ndl = (int32_t*)take(ni4);
  w.dfl = (int32_t*)take(ni4);
  w.ra = (int32_t*)take(ni4);
  w.rb = (int32_t*)take(ni4);
  w.org = (int32_t*)take(ni4);
  w.rflag = (int32_t*)take(ni4);
  w.gidx = (int32_t*)take(ni4);
  w.K = (int32_t*)take(nm4);
  w.ndf = (int32_t*)take(nm4);
  w.nrot = (int32_t*)take(nm4);
  w.grp = (int32_t*)take(al((size_t)mmax * 12));
  w.rho = (double*)take(nm8);
  w.Wg = (double*)take(big);
  w.Qc = (double*)take(big);
  w.U = (double*)take(big);
  w.Out = (double*)take(big);
  Node* dnodes = (Node*)take(nodes_b);

  int rc = ELPA_OK;
  // the table lives in host memory owned by this call: wait for the copy
  if (!flat.empty() && (hipMemcpyAsync(dnodes, flat.data(), flat.size() * sizeof(Node),
                                       hipMemcpyHostToDevice, st) != hipSuccess ||
                        hipStreamSynchronize(st) != hipSuccess))
    rc = ELPA_ERR_DEVICE;
  if (rc == ELPA_OK)
    hipLaunchKernelGGL(k_init, dim3(grid_for(n * n)), dim3(256), 0, st, n, d, e, w.L, w.Q);
  std::vector<int32_t> Kh((size_t)mmax), Gh(3 * (size_t)mmax);
  for (int l = (int)lv.size() - 1; rc == ELPA_OK && l >= 0; --l) {
    const int64_t M = (int64_t)lv[l].size();
    int64_t smax = 0;
    for (const Node& x : lv[l]) smax = std::max(smax, x.hi - x.lo);
    const int64_t per = (smax + 255) / 256;
    const Node* nl = dnodes + first[l];
    const dim3 b256(256);
    hipLaunchKernelGGL(k_prep, dim3((unsigned)M), b256, 0, st, nl, n, e, w);
    hipLaunchKernelGGL(k_gather, dim3((unsigned)(M * smax)), b256, 0, st, nl, n, smax, w);
    hipLaunchKernelGGL(k_rotate, dim3((unsigned)(M * per)), b256, 0, st, nl, per, w);
    const int64_t per4 = (smax + 3) / 4;  // four roots (waves) per workgroup
    hipLaunchKernelGGL(k_secular, dim3((unsigned)(M * per4)), b256, 0, st, nl, per4, w);
    hipLaunchKernelGGL(k_zhat, dim3((unsigned)(M * per)), b256, 0, st, nl, per, w);
    hipLaunchKernelGGL(k_vec, dim3((unsigned)(M * smax)), b256, 0, st, nl, smax, w);
    hipLaunchKernelGGL(k_compress, dim3((unsigned)(M * smax)), b256, 0, st, nl, smax, w);
    if (smax <= kSmall) {
      hipLaunchKernelGGL(k_gemm_small, dim3((unsigned)M), b256, 0, st, nl, w);
    } else {
      if (hipMemcpyAsync(Kh.data(), w.K, (size_t)M * 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipMemcpyAsync(Gh.data(), w.grp, (size_t)M * 12, hipMemcpyDeviceToHost, st) !=
              hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess) {
        rc = ELPA_ERR_DEVICE;
        break;
      }
      std::lock_guard<std::mutex> lock(ebt::Handles::get().mu);
      rocblas_handle h = ebt::handle_for(st);
      if (!h) {
        rc = ELPA_ERR_DEVICE;
        break;
      }
      // Out[0:s1] = Qc[0:s1, groups 0,1] U[groups 0,1];
      // Out[s1:s] = Qc[s1:s, groups 1,2] U[groups 1,2]
      const auto N_ = rocblas_operation_none;
      for (int64_t mi = 0; mi < M && rc == ELPA_OK; ++mi) {
        const Node& x = lv[l][(size_t)mi];
        const int64_t s = x.hi - x.lo, s1 = x.mid - x.lo, K = Kh[(size_t)mi];
        const int64_t g0 = Gh[3 * (size_t)mi], g1 = Gh[3 * (size_t)mi + 1],
                      g2 = Gh[3 * (size_t)mi + 2];
        if (K == 0) continue;
        const double* Qc = w.Qc + x.woff;
        const double* U = w.U + x.woff;
        double* Out = w.Out + x.woff;
        bool ok = true;
        if (g0 + g1 > 0)
          ok = ebt::Blas<double>::gemm(h, N_, N_, s1, K, g0 + g1, 1.0, Qc, s, U, s, 0.0, Out, s) ==
               rocblas_status_success;
        else
          hipLaunchKernelGGL(k_zero, dim3(grid_for(s1 * K)), dim3(256), 0, st, Out, s, s1, K);
        if (g1 + g2 > 0)
          ok = ok && ebt::Blas<double>::gemm(h, N_, N_, s - s1, K, g1 + g2, 1.0, Qc + g0 * s + s1,
                                             s, U + g0, s, 0.0, Out + s1, s) ==
                         rocblas_status_success;
        else
          hipLaunchKernelGGL(k_zero, dim3(grid_for((s - s1) * K)), dim3(256), 0, st, Out + s1, s,
                             s - s1, K);
        if (!ok) rc = ELPA_ERR_DEVICE;
      }
    }
    hipLaunchKernelGGL(k_vals, dim3((unsigned)(M * per)), b256, 0, st, nl, per, w);
    hipLaunchKernelGGL(k_final, dim3((unsigned)(M * smax)), b256, 0, st, nl, n, smax, w);
    if (hipGetLastError() != hipSuccess) rc = ELPA_ERR_DEVICE;
  }
  if (rc == ELPA_OK) {
    if (nev > 0)
      hipLaunchKernelGGL(k_output<E>, dim3(grid_for(n * nev)), dim3(256), 0, st, n, nev,
                         (const double*)w.Q, Z, ldz);
    hipLaunchKernelGGL(k_lam, dim3(grid_for(n)), dim3(256), 0, st, n, (const double*)w.L, lam);
    if (hipGetLastError() != hipSuccess) rc = ELPA_ERR_DEVICE;
  }
  const hipError_t e2 = hipFreeAsync(ws, st);
  if (rc == ELPA_OK && e2 != hipSuccess) rc = ELPA_ERR_DEVICE;
  return rc;
}

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

}  // namespace edc

extern "C" int elpa_tridiag_eigh(int64_t n, int64_t nev, const double* d, const double* e,
                                 double* lam, void* Z, int64_t ldz, int32_t dtype, void* stream) {
  const size_t es = dtype == ELPA_R64 ? 8 : dtype == ELPA_R32 ? 4 : dtype == ELPA_C64 ? 16 : 0;
  if (es == 0) return ELPA_ERR_DTYPE;
  if (n < 0 || nev < 0 || nev > n || ldz < std::max<int64_t>(n, 1) || n > (int64_t)INT32_MAX)
    return ELPA_ERR_ARG;
  if (n == 0) return ELPA_OK;
  if (!d || !lam || (n > 1 && !e) || (nev > 0 && !Z)) return ELPA_ERR_ARG;
  if (!edc::aligned(d, 8) || !edc::aligned(lam, 8) || (e && !edc::aligned(e, 8)) ||
      (Z && !edc::aligned(Z, es)))
    return ELPA_ERR_ALIGN;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  switch (dtype) {
    case ELPA_R64: return edc::run<double>(n, nev, d, e, lam, (double*)Z, ldz, st);
    case ELPA_R32: return edc::run<float>(n, nev, d, e, lam, (float*)Z, ldz, st);
    default: return edc::run<ebt::zc>(n, nev, d, e, lam, (ebt::zc*)Z, ldz, st);
  }
}
