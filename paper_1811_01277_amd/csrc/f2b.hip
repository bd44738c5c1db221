// Full -> band reduction (C ABI in include/elpa_f2b.h; Kus et al., Sec. 2).
//
// Panel p: the m = n-p-nbw rows below the band of columns [p, p+nbw) get a
// Householder QR, one column at a time, spread over G workgroups of 256 rows
// each, two launches per column and no waiting between workgroups:
//   reflect(i): every workgroup sums the G partial norms of column p+i in a
//     fixed order and derives the same larfg result (tau, beta, scale); it
//     scales its rows of the column into V (zeros above the unit lead) and
//     writes its partial products conj(v)^T A[:, p+j] for the panel's later
//     columns;
//   update(i): every workgroup sums those partials in a fixed order, applies
//     the reflector to its rows of the later columns, writes beta and the
//     zeros of column p+i, and the partial norms of column p+i+1.
// The panel is then mirrored into the rows above (Hermitian storage), and the
// trailing matrix A22 = A[p+nbw:, p+nbw:] is updated from both sides with the
// panel's compact-WY product Q = I - V T V^H, T = M^{-1} diag(tau),
// M = I + diag(tau) striu(V^H V), in the symmetric two-sided form:
//   X = A22 V T,  Y = T^H (V^H X),  W = X - V Y / 2,
//   Q^H A22 Q = A22 - V W^H - W V^H   (one product with inner dimension 2k),
// as GEMMs and triangular solves on the matrix cores (rocBLAS).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "../../include/elpa_f2b.h"
#include "../../include/elpa_hh.h"
#include "wy_blas.h"

namespace ef2b {

using ebt::Blas;
using ebt::Num;
using ebt::zc;

__device__ __forceinline__ double conj_(double a) { return a; }
__device__ __forceinline__ zc conj_(zc a) { return zc{a.re, -a.im}; }
__device__ __forceinline__ double sub(double a, double b) { return a - b; }
__device__ __forceinline__ zc sub(zc a, zc b) { return zc{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ double abs2(double a) { return a * a; }
__device__ __forceinline__ double abs2(zc a) { return a.re * a.re + a.im * a.im; }
__device__ __forceinline__ double re(double a) { return a; }
__device__ __forceinline__ double re(zc a) { return a.re; }
__device__ __forceinline__ double im(double) { return 0.0; }
__device__ __forceinline__ double im(zc a) { return a.im; }
template <typename E>
__device__ __forceinline__ E from_re(double x) {
  if constexpr (std::is_same<E, double>::value)
    return x;
  else
    return zc{x, 0.0};
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int w = 32; w >= 1; w >>= 1) x += __shfl_xor(x, w, 64);
  return x;
}
__device__ __forceinline__ zc wave_sum(zc x) { return zc{wave_sum(x.re), wave_sum(x.im)}; }

constexpr int kRows = 256;  // panel rows per workgroup (one per thread)
constexpr int kMaxNb = 256;

// sum over the workgroup's threads (4 waves); every thread gets the total
template <typename T>
__device__ __forceinline__ T block_sum(T x, T* red) {
  x = wave_sum(x);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = x;
  __syncthreads();
  T t = red[0];
  for (int w = 1; w < (int)(blockDim.x >> 6); ++w) t = Num<T>::add(t, red[w]);
  return t;
}

// partial norms sum |A[r0+row, col]|^2 over the group's rows with row > i
template <typename E>
__global__ __launch_bounds__(kRows) void k_pnorm(const E* __restrict__ A, int64_t lda, int64_t r0,
                                                 int64_t col, int64_t m, int64_t i,
                                                 double* __restrict__ pn) {
  __shared__ double red[4];
  const int64_t row = (int64_t)blockIdx.x * kRows + threadIdx.x;
  const double x = (row < m && row > i) ? abs2(A[r0 + row + col * lda]) : 0.0;
  const double t = block_sum(x, red);
  if (threadIdx.x == 0) pn[blockIdx.x] = t;
}

// larfg of column p+i from the partial norms, called by a whole wave: the
// lanes add the partials in a fixed order (lane l takes l, l+64, ...; then a
// butterfly), so every workgroup derives the same (tau, beta, scale)
template <typename E>
__device__ __forceinline__ void larfg_from(const E* __restrict__ A, int64_t lda, int64_t r0,
                                           int64_t p, int64_t i, int G,
                                           const double* __restrict__ pn, E* tau_out,
                                           double* beta_out, E* scale_out) {
  double part = 0.0;
  for (int g = (int)(threadIdx.x & 63); g < G; g += 64) part += pn[g];
  const double sum = wave_sum(part);
  const E alpha = A[r0 + i + (p + i) * lda];
  const double ar = re(alpha), ai = im(alpha);
  if (sum == 0.0 && ai == 0.0) {
    *tau_out = from_re<E>(0.0);
    *beta_out = ar;
    *scale_out = from_re<E>(1.0);
    return;
  }
  const double h = sqrt(ar * ar + ai * ai + sum);
  const double bt = (ar >= 0.0) ? -h : h;
  if constexpr (std::is_same<E, double>::value) {
    *tau_out = (bt - ar) / bt;
    *scale_out = 1.0 / (alpha - bt);
  } else {
    *tau_out = zc{(bt - ar) / bt, -ai / bt};
    const zc den{alpha.re - bt, alpha.im};
    const double dd = den.re * den.re + den.im * den.im;
    *scale_out = zc{den.re / dd, -den.im / dd};
  }
  *beta_out = bt;
}

template <typename E>
__global__ __launch_bounds__(kRows) void k_reflect(const E* __restrict__ A, int64_t lda,
                                                   int64_t r0, int64_t p, int64_t m, int64_t b,
                                                   int64_t i, int G, const double* __restrict__ pn,
                                                   E* __restrict__ V, int64_t ldv,
                                                   E* __restrict__ tau, E* __restrict__ pd) {
  __shared__ E sh[2];
  __shared__ E wred[kRows / 64][kMaxNb];
  if (threadIdx.x < 64) {
    E t, s;
    double beta;
    larfg_from(A, lda, r0, p, i, G, pn, &t, &beta, &s);
    if (threadIdx.x == 0) {
      sh[0] = t;
      sh[1] = s;
      if (blockIdx.x == 0) tau[p + i] = t;
    }
  }
  __syncthreads();
  const E sc = sh[1];
  const int64_t row = (int64_t)blockIdx.x * kRows + threadIdx.x;
  E v = from_re<E>(0.0);
  if (row < m) {
    if (row > i)
      v = Num<E>::mul(A[r0 + row + (p + i) * lda], sc);
    else if (row == i)
      v = from_re<E>(1.0);
    V[r0 + row + (p + i) * ldv] = v;  // zeros above the unit lead
  }
  // partial products conj(v)^T A[:, p+j]: every wave reduces all columns with
  // shuffles (no barrier between columns, so their loads overlap), then the
  // four waves' sums are added in a fixed order
  const E cv = conj_(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool own = row < m && row >= i;
  // eight columns' values loaded before any is reduced, so their loads are
  // in flight together
  constexpr int CH = 8;
  for (int64_t j0 = i + 1; j0 < b; j0 += CH) {
    E x[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u)
      x[u] = (own && j0 + u < b) ? A[r0 + row + (p + j0 + u) * lda] : from_re<E>(0.0);
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const E t = wave_sum(Num<E>::mul(cv, x[u]));
      if (lane == 0 && j0 + u < b) wred[wave][j0 + u] = t;
    }
  }
  __syncthreads();
  for (int64_t j = i + 1 + threadIdx.x; j < b; j += blockDim.x) {
    E t = wred[0][j];
    for (int w = 1; w < kRows / 64; ++w) t = Num<E>::add(t, wred[w][j]);
    pd[(int64_t)blockIdx.x * b + j] = t;
  }
}

template <typename E>
__global__ __launch_bounds__(kRows) void k_update(E* __restrict__ A, int64_t lda, int64_t r0,
                                                  int64_t p, int64_t m, int64_t b, int64_t i,
                                                  int G, const E* __restrict__ V, int64_t ldv,
                                                  const E* __restrict__ tau,
                                                  const double* __restrict__ pn_in,
                                                  const E* __restrict__ pd,
                                                  double* __restrict__ pn_out, int64_t k) {
  __shared__ E coef[kMaxNb];
  __shared__ double shb;
  __shared__ double red[4];
  const E ct = conj_(tau[p + i]);
  // coef[j] = conj(tau) sum_g pd[g][j]: one wave per column, lanes over the
  // partials in a fixed order
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t j = i + 1 + wave; j < b; j += kRows / 64) {
    E w = from_re<E>(0.0);
    for (int g = lane; g < G; g += 64) w = Num<E>::add(w, pd[(int64_t)g * b + j]);
    w = wave_sum(w);
    if (lane == 0) coef[j] = Num<E>::mul(ct, w);
  }
  if (threadIdx.x < 64) {
    E t, s;
    double beta;
    larfg_from(A, lda, r0, p, i, G, pn_in, &t, &beta, &s);
    if (threadIdx.x == 0) shb = beta;
  }
  __syncthreads();
  const int64_t row = (int64_t)blockIdx.x * kRows + threadIdx.x;
  if (row < m && row >= i) {
    const E v = (row == i) ? from_re<E>(1.0) : V[r0 + row + (p + i) * ldv];
    // eight columns loaded before any is written back: the stores could
    // alias the next loads as far as the compiler knows, which would
    // otherwise serialise every column's load behind the previous store
    constexpr int CH = 8;
    for (int64_t j0 = i + 1; j0 < b; j0 += CH) {
      E a[CH];
#pragma unroll
      for (int u = 0; u < CH; ++u)
        if (j0 + u < b) a[u] = A[r0 + row + (p + j0 + u) * lda];
#pragma unroll
      for (int u = 0; u < CH; ++u)
        if (j0 + u < b) A[r0 + row + (p + j0 + u) * lda] = sub(a[u], Num<E>::mul(v, coef[j0 + u]));
    }
    A[r0 + row + (p + i) * lda] = (row == i) ? from_re<E>(shb) : from_re<E>(0.0);
  }
  if (i + 1 < k) {  // partial norms of the next column, rows > i+1
    const double x = (row < m && row > i + 1) ? abs2(A[r0 + row + (p + i + 1) * lda]) : 0.0;
    const double t = block_sum(x, red);
    if (threadIdx.x == 0) pn_out[blockIdx.x] = t;
  }
}

// A[p+j, r0+row] = conj(A[r0+row, p+j]) for the panel
template <typename E>
__global__ __launch_bounds__(256) void k_mirror(E* __restrict__ A, int64_t lda, int64_t r0,
                                                int64_t p, int64_t m, int64_t b) {
  const int64_t j = blockIdx.y;
  for (int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; row < m;
       row += (int64_t)gridDim.x * blockDim.x)
    A[p + j + (r0 + row) * lda] = conj_(A[r0 + row + (p + j) * lda]);
}

// W (rows x cols, ld) scaled: by_rows: W[r, c] *= conj(tau[r]); else W[r, c] *= tau[c]
template <typename E>
__global__ __launch_bounds__(256) void k_scale(E* __restrict__ W, int64_t ld, int64_t rows,
                                               int64_t cols, const E* __restrict__ tau,
                                               bool by_rows) {
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e % rows, c = e / rows;
    E& w = W[r + c * ld];
    w = Num<E>::mul(by_rows ? conj_(tau[r]) : tau[c], w);
  }
}

template <typename E>
int run(int64_t n, int64_t b, E* A, int64_t lda, E* V, int64_t ldv, E* tau, hipStream_t st) {
  using S = typename std::conditional<std::is_same<E, float>::value, float, double>::type;
  const size_t es = sizeof(E);
  const int64_t mmax = n - b;
  const int Gmax = (int)((mmax + kRows - 1) / kRows);
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  size_t part_e = 0;  // the largest set of K-chunk partial products over the panels
  for (int64_t p = 0; p + b < n; p += b) {
    const int64_t m = n - p - b, k = std::min(b, m);
    part_e = std::max(part_e, (size_t)ebt::ksplit(m, k, k, es) * k * k);
  }
  const size_t off_pn = 0, off_pd = off_pn + al(2 * Gmax * sizeof(double) + 512),
               off_g = off_pd + al((size_t)Gmax * b * es), off_m = off_g + al((size_t)b * b * es),
               off_w1 = off_m + al((size_t)b * b * es),
               off_w2 = off_w1 + al((size_t)2 * b * mmax * es),
               off_part = off_w2 + al((size_t)2 * mmax * b * es), total = off_part + al(part_e * es);
  char* ws = nullptr;
  if (hipMallocAsync((void**)&ws, total, st) != hipSuccess) return ELPA_ERR_NOMEM;
  double* pn0 = (double*)(ws + off_pn);
  double* pn1 = pn0 + Gmax;
  E* pd = (E*)(ws + off_pd);
  E* Gm = (E*)(ws + off_g);
  E* M = (E*)(ws + off_m);
  E* W1 = (E*)(ws + off_w1);
  E* W2 = (E*)(ws + off_w2);
  E* part = (E*)(ws + off_part);
  int rc = ELPA_OK;
  {
    std::lock_guard<std::mutex> lock(ebt::Handles::get().mu);
    rocblas_handle h = ebt::handle_for(st);
    if (!h) rc = ELPA_ERR_DEVICE;
    const auto N_ = rocblas_operation_none;
    const auto C_ = Blas<E>::adj;
    for (int64_t p = 0; rc == ELPA_OK && p + b < n; p += b) {
      const int64_t r0 = p + b, m = n - r0, k = std::min(b, m);
      const int G = (int)((m + kRows - 1) / kRows);
      double* pa = pn0;
      double* pb = pn1;
      hipLaunchKernelGGL(k_pnorm<E>, dim3(G), dim3(kRows), 0, st, (const E*)A, lda, r0, p, m,
                         (int64_t)0, pa);
      for (int64_t i = 0; i < k; ++i) {
        hipLaunchKernelGGL(k_reflect<E>, dim3(G), dim3(kRows), 0, st, (const E*)A, lda, r0, p, m,
                           b, i, G, (const double*)pa, V, ldv, tau, pd);
        hipLaunchKernelGGL(k_update<E>, dim3(G), dim3(kRows), 0, st, A, lda, r0, p, m, b, i, G,
                           (const E*)V, ldv, (const E*)tau, (const double*)pa, (const E*)pd, pb,
                           k);
        std::swap(pa, pb);
      }
      hipLaunchKernelGGL(k_mirror<E>, dim3((unsigned)std::min<int64_t>((m + 255) / 256, 1024),
                                           (unsigned)b),
                         dim3(256), 0, st, A, lda, r0, p, m, b);
      // trailing update with the panel's k reflectors
      const E* Vp = V + r0 + p * ldv;
      E* A22 = A + r0 + r0 * lda;
      const E* tp = tau + p;
      bool ok = ebt::gemm_adj_splitk<E, S>(h, k, k, m, Vp, ldv, Vp, ldv,
                                           ebt::ksplit(m, k, k, es), part, nullptr, Gm, st);
      if (ok)
        hipLaunchKernelGGL(ebt::k_unit_tri<E>, dim3((unsigned)((k * k + 255) / 256)), dim3(256),
                           0, st, (const E*)Gm, tp, k, M);
      // X = A22 V T (T = M^{-1} diag(tau)) into the W half of P = [V | W]
      E* Pv = W1;
      E* Pw = W1 + m * k;
      E* Rw = W2;
      E* Rv = W2 + m * k;
      const auto D2D = hipMemcpyDeviceToDevice;
      ok = ok && hipMemcpy2DAsync(Pv, (size_t)m * es, Vp, (size_t)ldv * es, (size_t)m * es,
                                  (size_t)k, D2D, st) == hipSuccess;
      ok = ok && hipMemcpy2DAsync(Rv, (size_t)m * es, Vp, (size_t)ldv * es, (size_t)m * es,
                                  (size_t)k, D2D, st) == hipSuccess;
      ok = ok && Blas<E>::gemm(h, N_, N_, m, k, m, S(1), A22, lda, Vp, ldv, S(0), Pw, m) ==
                     rocblas_status_success;
      ok = ok && Blas<E>::trsm(h, rocblas_side_right, N_, m, k, M, k, Pw, m) ==
                     rocblas_status_success;
      if (ok)
        hipLaunchKernelGGL(k_scale<E>, dim3((unsigned)std::min<int64_t>((k * m + 255) / 256, 4096)),
                           dim3(256), 0, st, Pw, m, m, k, tp, false);
      // Y = T^H V^H X = diag(conj tau) M^{-H} (V^H X), k x k (in Gm)
      ok = ok && ebt::gemm_adj_splitk<E, S>(h, k, k, m, Vp, ldv, Pw, m, ebt::ksplit(m, k, k, es),
                                            part, nullptr, Gm, st);
      ok = ok && Blas<E>::trsm(h, rocblas_side_left, C_, k, k, M, k, Gm, k) ==
                     rocblas_status_success;
      if (ok)
        hipLaunchKernelGGL(k_scale<E>, dim3((unsigned)((k * k + 255) / 256)), dim3(256), 0, st,
                           Gm, k, k, k, tp, true);
      // W = X - V Y / 2, so that Q^H A22 Q = A22 - V W^H - W V^H
      ok = ok && Blas<E>::gemm(h, N_, N_, m, k, k, S(-0.5), Vp, ldv, Gm, k, S(1), Pw, m) ==
                     rocblas_status_success;
      ok = ok && hipMemcpyAsync(Rw, Pw, (size_t)m * k * es, D2D, st) == hipSuccess;
      // A22 -= [V W] [W V]^H: one rank-2k product over both triangles
      ok = ok && Blas<E>::gemm(h, N_, C_, m, m, 2 * k, S(-1), W1, m, W2, m, S(1), A22, lda) ==
                     rocblas_status_success;
      if (!ok || hipGetLastError() != hipSuccess) rc = ELPA_ERR_DEVICE;
    }
  }
  const hipError_t e2 = hipFreeAsync(ws, st);
  if (rc == ELPA_OK && e2 != hipSuccess) rc = ELPA_ERR_DEVICE;
  return rc;
}

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

}  // namespace ef2b

extern "C" int elpa_full_to_band(int64_t n, int64_t nbw, void* A, int64_t lda, void* V,
                                 int64_t ldv, void* tau, int32_t dtype, void* stream) {
  if (dtype != ELPA_R64 && dtype != ELPA_C64) return ELPA_ERR_DTYPE;
  if (n < 1 || nbw < 1 || nbw > ef2b::kMaxNb || lda < n || ldv < n) return ELPA_ERR_ARG;
  if (!A) return ELPA_ERR_ARG;
  if (n <= nbw) return ELPA_OK;
  if (!V || !tau) return ELPA_ERR_ARG;
  const size_t es = dtype == ELPA_C64 ? 16 : 8;
  if (!ef2b::aligned(A, es) || !ef2b::aligned(V, es) || !ef2b::aligned(tau, es))
    return ELPA_ERR_ALIGN;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (dtype == ELPA_R64)
    return ef2b::run<double>(n, nbw, (double*)A, lda, (double*)V, ldv, (double*)tau, st);
  return ef2b::run<ebt::zc>(n, nbw, (ebt::zc*)A, lda, (ebt::zc*)V, ldv, (ebt::zc*)tau, st);
}
