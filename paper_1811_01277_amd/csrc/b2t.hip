// Band -> tridiagonal reduction by bulge chasing (C ABI in
// include/elpa_b2t.h; Kus et al., Sec. 2), one column per chase step, with
// the reflectors written in the slot layout of the tridiagonal -> band
// back-transformation.
//
// Schedule.  Chase step (s, j) (row r = s+1+j*nbw, length L <= nbw) reads and
// writes only entries of the square [r-nbw, r+L+nbw)^2 that lie in rows
// [r, r+L) or in columns [r, r+L).  A step (s+1, j') with j' <= j-3 stays
// within indices up to r-nbw, and meets index r-nbw only in rows and columns
// below r, so it shares no entry with (s, j); steps further apart share none
// either.  So with the launch index
//   t(s, j) = j + 3 s
// every pair that shares entries runs in launches ordered as in the
// sequential reduction (sweep by sweep, step by step), and the steps of one
// launch (same t, distinct s) touch disjoint entries.  One workgroup per step;
// kernel boundaries order the launches.  There is no waiting between
// workgroups.
//
// A step: the reflector from column c (= s for j = 0, else r - nbw), rows
// [r, r+L) (LAPACK's larfg convention), then the left update of rows
// [r, r+L) over the window's columns (one wave per column, lanes over rows)
// and the right update of columns [r, r+L) over the window's rows (one
// thread per row), then the eliminated entries written exactly.  The step is
// bound by memory latency, so both updates issue a chunk of independent
// loads before using any of them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "../../include/elpa_b2t.h"
#include "../../include/elpa_hh.h"
#include "hh_common.h"

namespace eb2t {

using ehh::z64;

// scalar operations on double / complex double
__device__ __forceinline__ double conj_(double a) { return a; }
__device__ __forceinline__ z64 conj_(z64 a) { return z64{a.re, -a.im}; }
__device__ __forceinline__ double mul(double a, double b) { return a * b; }
__device__ __forceinline__ z64 mul(z64 a, z64 b) {
  return z64{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ double add(double a, double b) { return a + b; }
__device__ __forceinline__ z64 add(z64 a, z64 b) { return z64{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ double sub(double a, double b) { return a - b; }
__device__ __forceinline__ z64 sub(z64 a, z64 b) { return z64{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ double abs2(double a) { return a * a; }
__device__ __forceinline__ double abs2(z64 a) { return a.re * a.re + a.im * a.im; }
__device__ __forceinline__ double re(double a) { return a; }
__device__ __forceinline__ double re(z64 a) { return a.re; }
__device__ __forceinline__ double im(double) { return 0.0; }
__device__ __forceinline__ double im(z64 a) { return a.im; }
template <typename E>
__device__ __forceinline__ E from_re(double x) {
  if constexpr (std::is_same<E, double>::value)
    return x;
  else
    return z64{x, 0.0};
}
template <typename E>
__device__ __forceinline__ E zero() {
  return from_re<E>(0.0);
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int w = 32; w >= 1; w >>= 1) x += __shfl_xor(x, w, 64);
  return x;
}
__device__ __forceinline__ z64 wave_sum(z64 x) { return z64{wave_sum(x.re), wave_sum(x.im)}; }

constexpr int kMaxNb = 512;
// Launch t runs the steps (s, t - kLag s): two steps of one launch touch
// disjoint entries (the later sweep only rows and columns below r - nb, the
// earlier one only from r on, sharing index r - nb in different entries).
constexpr int64_t kLag = 3;

// one launch: the steps (s, t - kLag s) for s = s_lo .. s_lo + gridDim.x - 1, one
// 512-thread workgroup (8 waves) per step
template <typename E>
__global__ __launch_bounds__(512) void k_chase(E* __restrict__ A, int64_t lda, int64_t n,
                                               int64_t nb, int64_t t, int64_t s_lo,
                                               E* __restrict__ hh, E* __restrict__ tau) {
  __shared__ E v[kMaxNb];
  __shared__ double part[8];
  __shared__ E sh_tau, sh_sc;
  __shared__ double sh_beta;
  const int64_t s = s_lo + blockIdx.x;
  const int64_t j = t - kLag * s;
  const int64_t r = s + 1 + j * nb;
  const int64_t L = (nb < n - r) ? nb : n - r;
  const int64_t c = (j == 0) ? s : r - nb;
  const int64_t lo = (r - nb > 0) ? r - nb : 0;
  const int64_t hi = (r + L + nb < n) ? r + L + nb : n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  auto at = [&](int64_t i, int64_t k) -> E& { return A[i + k * lda]; };

  // reflector: x = A[r .. r+L, c]
  double ss = 0.0;
  for (int64_t i = tid; i < L; i += blockDim.x) {
    const E x = at(r + i, c);
    v[i] = x;
    if (i >= 1) ss += abs2(x);
  }
  ss = wave_sum(ss);
  if (lane == 0) part[wave] = ss;
  __syncthreads();
  if (tid == 0) {
    double sum = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) sum += part[w];
    const E alpha = v[0];
    const double ar = re(alpha), ai = im(alpha);
    if (sum == 0.0 && ai == 0.0) {
      sh_tau = zero<E>();
      sh_beta = ar;
      part[0] = 0.0;  // no scaling needed
    } else {
      const double h = sqrt(ar * ar + ai * ai + sum);
      const double bt = (ar >= 0.0) ? -h : h;
      if constexpr (std::is_same<E, double>::value)
        sh_tau = (bt - ar) / bt;
      else
        sh_tau = z64{(bt - ar) / bt, -ai / bt};
      sh_beta = bt;
      part[0] = 1.0;
      // scale 1 / (alpha - beta)
      const E den = sub(alpha, from_re<E>(bt));
      if constexpr (std::is_same<E, double>::value) {
        sh_sc = 1.0 / den;
      } else {
        const double dd = den.re * den.re + den.im * den.im;
        sh_sc = z64{den.re / dd, -den.im / dd};
      }
    }
  }
  __syncthreads();
  const E tv = sh_tau;
  const bool act = part[0] != 0.0;
  {
    // v <- (1, x[1:] / (alpha - beta)); with tau = 0 the tail is already zero
    const E sc = sh_sc;
    for (int64_t i = tid; i < L; i += blockDim.x)
      v[i] = (i == 0) ? from_re<E>(1.0) : (act ? mul(v[i], sc) : v[i]);
  }
  __syncthreads();

  if (act) {
    // left: rows [r, r+L) of columns [lo, hi) <- H^H rows, H^H = I - conj(tau) v v^H.
    // A wave takes columns lo+wave, lo+wave+NW, ...; with L <= 64 a lane holds
    // one row, and the values of CH columns are loaded before any is used,
    // so CH loads are in flight at once.
    const E ct = conj_(tv);
    const int NW = (int)(blockDim.x >> 6);
    if (L <= 64) {
      constexpr int CH = 8;
      const E vl = lane < L ? v[lane] : zero<E>();
      const E cvl = conj_(vl);
      for (int64_t k0 = lo + wave; k0 < hi; k0 += (int64_t)NW * CH) {
        E x[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
          const int64_t k = k0 + (int64_t)NW * u;
          x[u] = (k < hi && lane < L) ? at(r + lane, k) : zero<E>();
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
          const int64_t k = k0 + (int64_t)NW * u;
          const E w = mul(ct, wave_sum(mul(cvl, x[u])));
          if (k < hi && lane < L) at(r + lane, k) = sub(x[u], mul(vl, w));
        }
      }
    } else {
      for (int64_t k = lo + wave; k < hi; k += NW) {
        E acc = zero<E>();
        for (int64_t i = lane; i < L; i += 64) acc = add(acc, mul(conj_(v[i]), at(r + i, k)));
        const E w = mul(ct, wave_sum(acc));
        for (int64_t i = lane; i < L; i += 64) at(r + i, k) = sub(at(r + i, k), mul(v[i], w));
      }
    }
    __syncthreads();
    // right: columns [r, r+L) of rows [lo, hi) <- cols H, H = I - tau v v^H.
    // Four adjacent threads per row, each with QC consecutive columns of every
    // 4 QC; their partial products are combined by lane shuffles (all four get
    // the same sum in the same order), and every thread updates the values it
    // loaded.  Rows with L > 4 QC reload their values for the update.
    constexpr int QC = 16;
    const int part4 = tid & 3;
    const int64_t rows_per_pass = blockDim.x >> 2;
    for (int64_t i0 = lo; i0 < hi; i0 += rows_per_pass) {
      const int64_t i = i0 + (tid >> 2);
      const bool row_ok = i < hi;
      E y[QC];
      E acc = zero<E>();
      for (int64_t q0 = 0; q0 < L; q0 += 4 * QC) {
        const int64_t qb = q0 + (int64_t)part4 * QC;
#pragma unroll
        for (int u = 0; u < QC; ++u)
          y[u] = (row_ok && qb + u < L) ? at(i, r + qb + u) : zero<E>();
#pragma unroll
        for (int u = 0; u < QC; ++u)
          if (qb + u < L) acc = add(acc, mul(y[u], v[qb + u]));
      }
      // sum over the four threads of the row (lanes 4m .. 4m+3 of one wave)
      E tot = acc;
      if constexpr (std::is_same<E, double>::value) {
        tot = tot + __shfl_xor(tot, 1, 64);
        tot = tot + __shfl_xor(tot, 2, 64);
      } else {
        tot = z64{tot.re + __shfl_xor(tot.re, 1, 64), tot.im + __shfl_xor(tot.im, 1, 64)};
        tot = z64{tot.re + __shfl_xor(tot.re, 2, 64), tot.im + __shfl_xor(tot.im, 2, 64)};
      }
      const E w = mul(tot, tv);
      if (L <= 4 * QC) {
        const int64_t qb = (int64_t)part4 * QC;
#pragma unroll
        for (int u = 0; u < QC; ++u)
          if (row_ok && qb + u < L) at(i, r + qb + u) = sub(y[u], mul(w, conj_(v[qb + u])));
      } else {
        for (int64_t q0 = 0; q0 < L; q0 += 4 * QC) {
          const int64_t qb = q0 + (int64_t)part4 * QC;
#pragma unroll
          for (int u = 0; u < QC; ++u)
            if (row_ok && qb + u < L)
              at(i, r + qb + u) = sub(at(i, r + qb + u), mul(w, conj_(v[qb + u])));
        }
      }
    }
  }
  __syncthreads();
  // eliminated entries, the reflector in its slot
  const E beta = from_re<E>(sh_beta);
  const int64_t slot = ehh::slot_offset(n, nb, s) + j;
  E* __restrict__ dst = hh + slot * nb;
  for (int64_t i = tid; i < nb; i += blockDim.x) {
    if (i < L) {
      const E z = (i == 0) ? beta : zero<E>();
      at(r + i, c) = z;
      at(c, r + i) = z;
    }
    dst[i] = (i < L) ? v[i] : zero<E>();
  }
  if (tid == 0) tau[slot] = tv;
}

// Real band, nb <= 64: the same steps on the lower triangle only, every value
// a step touches held in registers (the upper triangle is rebuilt at the end
// from the tridiagonal result).  A step (s, j) with H = I - tau v v^T on the
// indices [r, r+L) changes three lower-triangle blocks:
//   R = rows [r, r+L) x columns [c0, r)   <- H R   (c0 = s for j = 0: the
//       columns left of s are already reduced and zero in these rows; else
//       r - nb, the bulge columns)
//   D = rows and columns [r, r+L)         <- H D H (symmetric; with y = D v,
//       mu = v^T y and w = tau y - tau^2 mu / 2 v: D <- D - w v^T - v w^T)
//   C = rows [r+L, hi) x columns [r, r+L) <- C H   (hi = min(r+L+nb, n))
// Lane i of every wave holds row i of each block, wave w of the NW waves the
// columns w, w+NW, ..., so each block is one coalesced load per column, all
// issued before any value is used, and one store.  Column sums (v^T R, the
// strictly-lower part of D^T v) are wave reductions; row sums (the lower part
// of D v, C v) add the waves' partial sums through LDS.  Two barriers per
// step.  With eight waves each wave's chain of column reductions is half as
// long as with four (n = 20000, nbw = 64: 0.80 s against 1.04 s; sixteen
// waves gave 0.81 s).  The
// lower-triangle entries the steps touch are a subset of the two-sided form's,
// so the launch schedule's disjointness holds unchanged.
template <int NW>
__global__ __launch_bounds__(64 * NW) void k_chase_reg(double* __restrict__ A, int64_t lda, int64_t n,
                                                   int64_t nb, int64_t t, int64_t s_lo,
                                                   double* __restrict__ hh,
                                                   double* __restrict__ tau) {
  __shared__ double vs[64], ys2[64], py[NW][64], pu[NW][64];
  __shared__ double sh_tau;
  const int64_t s = s_lo + blockIdx.x;
  const int64_t j = t - kLag * s;
  const int64_t r = s + 1 + j * nb;
  const int L = (int)((nb < n - r) ? nb : n - r);
  const int64_t c0 = (j == 0) ? s : r - nb;
  const int nR = (int)(r - c0);                       // 1 for j = 0, else nb
  const int nC = (int)(((r + L + nb < n) ? r + L + nb : n) - r - L);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  auto at = [&](int64_t i, int64_t k) -> double& { return A[i + k * lda]; };

  constexpr int NQ = 64 / NW;  // columns per wave
  double xr[NQ], xd[NQ], xc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int k = wave + NW * q;
    xr[q] = (lane < L && k < nR) ? at(r + lane, c0 + k) : 0.0;
    xd[q] = (lane < L && k < L && lane >= k) ? at(r + lane, r + k) : 0.0;
    xc[q] = (lane < nC && k < L) ? at(r + L + lane, r + k) : 0.0;
  }
  // reflector from column 0 of R (column c0, the column this step reduces;
  // wave 0's first column)
  if (wave == 0) {
    const double x = xr[0];
    const double ss = wave_sum(lane >= 1 ? x * x : 0.0);
    const double alpha = __shfl(x, 0, 64);
    double tv = 0.0, beta = alpha, sc = 0.0;
    if (ss != 0.0) {
      const double h = sqrt(alpha * alpha + ss);
      beta = alpha >= 0.0 ? -h : h;
      tv = (beta - alpha) / beta;
      sc = 1.0 / (alpha - beta);
    }
    vs[lane] = lane == 0 ? 1.0 : (lane < L ? x * sc : 0.0);
    xr[0] = lane == 0 ? beta : 0.0;   // the reduced column, exactly
    if (lane == 0) sh_tau = tv;
  }
  __syncthreads();
  const double tv = sh_tau;
  const double vl = vs[lane];
  double vk[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) vk[q] = vs[wave + NW * q];
  if (tv != 0.0) {
    // column sums: v^T R (R's update) and the strictly lower part of D^T v;
    // row sums: the lower part of D v and C v, per wave
    double wr[NQ];
    double ry = 0.0, ru = 0.0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int k = wave + NW * q;
      wr[q] = (k >= 1) ? tv * wave_sum(vl * xr[q]) : 0.0;
      const double cs = wave_sum(lane > k ? vl * xd[q] : 0.0);
      if (lane == 0) ys2[k] = cs;
      ry += xd[q] * vk[q];
      ru += xc[q] * vk[q];
    }
    py[wave][lane] = ry;
    pu[wave][lane] = ru;
    __syncthreads();
    // y = D v, u = tau C v, mu = v^T y, w = tau y - tau^2 mu / 2 v (every
    // wave forms the values of its own rows and columns)
    double yl = ys2[lane], us = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      yl += py[w][lane];
      us += pu[w][lane];
    }
    const double ul = tv * us;
    const double mu = wave_sum(vl * yl);
    const double h2 = 0.5 * tv * tv * mu;
    const double wl = tv * yl - h2 * vl;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int k = wave + NW * q;
      double yk = ys2[k];
#pragma unroll
      for (int w = 0; w < NW; ++w) yk += py[w][k];
      const double wk = tv * yk - h2 * vk[q];
      if (k >= 1) xr[q] -= vl * wr[q];
      xd[q] -= wl * vk[q] + vl * wk;
      xc[q] -= ul * vk[q];
    }
  }
  // store R, D (lower), C; the reflector in its slot
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int k = wave + NW * q;
    if (lane < L && k < nR) at(r + lane, c0 + k) = xr[q];
    if (lane < L && k < L && lane >= k) at(r + lane, r + k) = xd[q];
    if (lane < nC && k < L) at(r + L + lane, r + k) = xc[q];
  }
  const int64_t slot = ehh::slot_offset(n, nb, s) + j;
  if (tid < nb) hh[slot * nb + tid] = tid < L ? vs[tid] : 0.0;
  if (tid == 0) tau[slot] = tv;
}

// The upper triangle of the result (the register chase updates only the
// lower one): A[k-1, k] = e[k-1], zeros above it up to 2 nb rows.
__global__ __launch_bounds__(256) void k_upper_out(double* __restrict__ A, int64_t lda,
                                                   int64_t n, int64_t nb,
                                                   const double* __restrict__ e) {
  const int64_t k = (int64_t)blockIdx.x + 1;   // columns 1 .. n-1
  const int64_t span = 2 * nb;
  for (int64_t q = threadIdx.x; q < span; q += blockDim.x) {
    const int64_t i = k - 1 - q;
    if (i < 0) break;
    A[i + k * lda] = q == 0 ? e[k - 1] : 0.0;
  }
}

template <typename E>
__global__ __launch_bounds__(256) void k_diag_out(const E* __restrict__ A, int64_t lda,
                                                  int64_t n, double* __restrict__ d,
                                                  double* __restrict__ e) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    d[i] = re(A[i + i * lda]);
    if (i + 1 < n) e[i] = re(A[i + 1 + i * lda]);
  }
}

// J(s) = ceil((n-1-s)/nb)
inline int64_t steps_of(int64_t n, int64_t nb, int64_t s) { return (n - 1 - s + nb - 1) / nb; }

template <typename E>
int run(int64_t n, int64_t nb, E* A, int64_t lda, double* d, double* e, E* hh, E* tau,
        hipStream_t st) {
  // launches t = 0 .. T-1 with T = max_s (3 s + J(s)); the active sweeps of
  // launch t are s_lo(t) .. min(t / kLag, n - 2), s_lo the least s with
  // 3 s + J(s) > t (3 s + J(s) increases with s)
  int64_t T = 0;
  for (int64_t s = 0; s <= n - 2; ++s) T = std::max(T, kLag * s + steps_of(n, nb, s));
  // real bands up to 64 wide take the register, lower-triangle steps
  constexpr bool real = std::is_same<E, double>::value;
  const bool lower = real && nb <= 64;
  int64_t s_lo = 0;
  for (int64_t t = 0; t < T; ++t) {
    while (s_lo <= n - 2 && kLag * s_lo + steps_of(n, nb, s_lo) <= t) ++s_lo;
    const int64_t s_hi = std::min<int64_t>(t / kLag, n - 2);
    if (s_hi < s_lo) continue;
    if constexpr (real) {
      if (lower) {
        hipLaunchKernelGGL(k_chase_reg<8>, dim3((unsigned)(s_hi - s_lo + 1)), dim3(512), 0, st, A,
                           lda, n, nb, t, s_lo, hh, tau);
        continue;
      }
    }
    hipLaunchKernelGGL(k_chase<E>, dim3((unsigned)(s_hi - s_lo + 1)), dim3(512), 0, st, A, lda,
                       n, nb, t, s_lo, hh, tau);
  }
  const unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_diag_out<E>, dim3(g), dim3(256), 0, st, (const E*)A, lda, n, d, e);
  if constexpr (real) {
    if (lower && n > 1)
      hipLaunchKernelGGL(k_upper_out, dim3((unsigned)n - 1), dim3(256), 0, st, (double*)A, lda,
                         n, nb, (const double*)e);
  }
  return hipGetLastError() == hipSuccess ? ELPA_OK : ELPA_ERR_DEVICE;
}

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

}  // namespace eb2t

extern "C" int elpa_band_to_tridiag(int64_t n, int64_t nbw, void* A, int64_t lda, double* d,
                                    double* e, void* hh, void* tau, int32_t dtype,
                                    void* stream) {
  if (dtype != ELPA_R64 && dtype != ELPA_C64) return ELPA_ERR_DTYPE;
  if (n < 1 || nbw < 1 || nbw > eb2t::kMaxNb || lda < n) return ELPA_ERR_ARG;
  if (!A || !d || (n > 1 && (!e || !hh || !tau))) return ELPA_ERR_ARG;
  const size_t es = dtype == ELPA_C64 ? 16 : 8;
  if (!eb2t::aligned(A, es) || !eb2t::aligned(d, 8) || (n > 1 && (!eb2t::aligned(e, 8) ||
      !eb2t::aligned(hh, es) || !eb2t::aligned(tau, es))))
    return ELPA_ERR_ALIGN;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (dtype == ELPA_R64)
    return eb2t::run<double>(n, nbw, (double*)A, lda, d, e, (double*)hh, (double*)tau, st);
  return eb2t::run<ehh::z64>(n, nbw, (ehh::z64*)A, lda, d, e, (ehh::z64*)hh, (ehh::z64*)tau,
                             st);
}
