// Compact-WY building blocks on rocBLAS shared by the band -> full
// back-transformation and the full -> band reduction: element operations, the
// unit triangle M = I + diag(tau) striu(V^H V) whose inverse times diag(tau)
// is the compact-WY factor T (T^{-1} = diag(1/tau) + striu(V^H V)), a
// fixed-order sum of K-chunk partial products, rocBLAS wrappers per element
// type (the _64 entry points), one rocBLAS handle per device, and the split-K
// product A^H B for small outputs with long contractions.
#pragma once

#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <algorithm>
#include <cstdint>
#include <mutex>
#include <vector>

namespace ebt {

struct zc {
  double re, im;
};

template <typename E>
struct Num;
template <>
struct Num<double> {
  static __device__ __forceinline__ double zero() { return 0.0; }
  static __device__ __forceinline__ double one() { return 1.0; }
  static __device__ __forceinline__ double mul(double a, double b) { return a * b; }
  static __device__ __forceinline__ double add(double a, double b) { return a + b; }
};
template <>
struct Num<float> {
  static __device__ __forceinline__ float zero() { return 0.0f; }
  static __device__ __forceinline__ float one() { return 1.0f; }
  static __device__ __forceinline__ float mul(float a, float b) { return a * b; }
  static __device__ __forceinline__ float add(float a, float b) { return a + b; }
};
template <>
struct Num<zc> {
  static __device__ __forceinline__ zc zero() { return {0.0, 0.0}; }
  static __device__ __forceinline__ zc one() { return {1.0, 0.0}; }
  static __device__ __forceinline__ zc mul(zc a, zc b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
  }
  static __device__ __forceinline__ zc add(zc a, zc b) { return {a.re + b.re, a.im + b.im}; }
};

// M = I + diag(tau) striu(G) (wb x wb, column major), G = V^H V (ld wb).
template <typename E>
__global__ __launch_bounds__(256) void k_unit_tri(const E* __restrict__ G,
                                                  const E* __restrict__ tau, int64_t wb,
                                                  E* __restrict__ M) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= wb * wb) return;
  const int64_t j = e % wb, i = e / wb;
  M[e] = j < i ? Num<E>::mul(tau[j], G[e]) : (j == i ? Num<E>::one() : Num<E>::zero());
}

// out[e] = scale(e) * sum_s part[s][e] over cnt partial products of `total`
// elements each (fixed order: the same bits on every call); scale is tau[e %
// wb] when tau is given (the row scaling of W), else 1.
template <typename E>
__global__ __launch_bounds__(256) void k_sum_parts(const E* __restrict__ part, int64_t cnt,
                                                   int64_t total, const E* __restrict__ tau,
                                                   int64_t wb, E* __restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    E acc = part[e];
    for (int64_t k = 1; k < cnt; ++k) acc = Num<E>::add(acc, part[k * total + e]);
    out[e] = tau ? Num<E>::mul(tau[e % wb], acc) : acc;
  }
}

// rocBLAS per element type
template <typename E>
struct Blas;
template <>
struct Blas<double> {
  static rocblas_status gemm(rocblas_handle h, rocblas_operation ta, rocblas_operation tb,
                             int64_t m, int64_t n, int64_t k, double alpha, const double* A,
                             int64_t lda, const double* B, int64_t ldb, double beta, double* C,
                             int64_t ldc) {
    return rocblas_dgemm_64(h, ta, tb, m, n, k, &alpha, A, lda, B, ldb, &beta, C, ldc);
  }
  static rocblas_status gemm_sb(rocblas_handle h, rocblas_operation ta, rocblas_operation tb,
                                int64_t m, int64_t n, int64_t k, double alpha, const double* A,
                                int64_t lda, int64_t sa, const double* B, int64_t ldb, int64_t sb,
                                double beta, double* C, int64_t ldc, int64_t sc, int64_t cnt) {
    return rocblas_dgemm_strided_batched_64(h, ta, tb, m, n, k, &alpha, A, lda, sa, B, ldb, sb,
                                            &beta, C, ldc, sc, cnt);
  }
  static rocblas_status trsm(rocblas_handle h, rocblas_side side, rocblas_operation op, int64_t m,
                             int64_t n, const double* A, int64_t lda, double* B, int64_t ldb) {
    const double one = 1.0;
    return rocblas_dtrsm_64(h, side, rocblas_fill_upper, op, rocblas_diagonal_unit, m, n, &one, A,
                            lda, B, ldb);
  }
  static constexpr rocblas_operation adj = rocblas_operation_transpose;
};
template <>
struct Blas<float> {
  static rocblas_status gemm(rocblas_handle h, rocblas_operation ta, rocblas_operation tb,
                             int64_t m, int64_t n, int64_t k, float alpha, const float* A,
                             int64_t lda, const float* B, int64_t ldb, float beta, float* C,
                             int64_t ldc) {
    return rocblas_sgemm_64(h, ta, tb, m, n, k, &alpha, A, lda, B, ldb, &beta, C, ldc);
  }
  static rocblas_status gemm_sb(rocblas_handle h, rocblas_operation ta, rocblas_operation tb,
                                int64_t m, int64_t n, int64_t k, float alpha, const float* A,
                                int64_t lda, int64_t sa, const float* B, int64_t ldb, int64_t sb,
                                float beta, float* C, int64_t ldc, int64_t sc, int64_t cnt) {
    return rocblas_sgemm_strided_batched_64(h, ta, tb, m, n, k, &alpha, A, lda, sa, B, ldb, sb,
                                            &beta, C, ldc, sc, cnt);
  }
  static rocblas_status trsm(rocblas_handle h, rocblas_side side, rocblas_operation op, int64_t m,
                             int64_t n, const float* A, int64_t lda, float* B, int64_t ldb) {
    const float one = 1.0f;
    return rocblas_strsm_64(h, side, rocblas_fill_upper, op, rocblas_diagonal_unit, m, n, &one, A,
                            lda, B, ldb);
  }
  static constexpr rocblas_operation adj = rocblas_operation_transpose;
};
template <>
struct Blas<zc> {
  static rocblas_status gemm(rocblas_handle h, rocblas_operation ta, rocblas_operation tb,
                             int64_t m, int64_t n, int64_t k, double alpha, const zc* A,
                             int64_t lda, const zc* B, int64_t ldb, double beta, zc* C,
                             int64_t ldc) {
    const rocblas_double_complex a{alpha, 0.0}, b{beta, 0.0};
    return rocblas_zgemm_64(h, ta, tb, m, n, k, &a, (const rocblas_double_complex*)A, lda,
                            (const rocblas_double_complex*)B, ldb, &b,
                            (rocblas_double_complex*)C, ldc);
  }
  static rocblas_status gemm_sb(rocblas_handle h, rocblas_operation ta, rocblas_operation tb,
                                int64_t m, int64_t n, int64_t k, double alpha, const zc* A,
                                int64_t lda, int64_t sa, const zc* B, int64_t ldb, int64_t sb,
                                double beta, zc* C, int64_t ldc, int64_t sc, int64_t cnt) {
    const rocblas_double_complex a{alpha, 0.0}, b{beta, 0.0};
    return rocblas_zgemm_strided_batched_64(h, ta, tb, m, n, k, &a,
                                            (const rocblas_double_complex*)A, lda, sa,
                                            (const rocblas_double_complex*)B, ldb, sb, &b,
                                            (rocblas_double_complex*)C, ldc, sc, cnt);
  }
  static rocblas_status trsm(rocblas_handle h, rocblas_side side, rocblas_operation op, int64_t m,
                             int64_t n, const zc* A, int64_t lda, zc* B, int64_t ldb) {
    const rocblas_double_complex one{1.0, 0.0};
    return rocblas_ztrsm_64(h, side, rocblas_fill_upper, op, rocblas_diagonal_unit, m, n, &one,
                            (const rocblas_double_complex*)A, lda, (rocblas_double_complex*)B,
                            ldb);
  }
  static constexpr rocblas_operation adj = rocblas_operation_conjugate_transpose;
};

// One rocBLAS handle per device; calls on a device are serialised (a handle
// holds one stream at a time).
struct Handles {
  std::mutex mu;
  std::vector<rocblas_handle> h;
  static Handles& get() {
    static Handles x;
    return x;
  }
};

// The rocBLAS handle of the current device, bound to stream st (call with
// Handles::get().mu held).
inline rocblas_handle handle_for(hipStream_t st) {
  Handles& H = Handles::get();
  int dev = 0;
  (void)hipGetDevice(&dev);
  if ((size_t)dev >= H.h.size()) H.h.resize((size_t)dev + 1, nullptr);
  if (!H.h[(size_t)dev] && rocblas_create_handle(&H.h[(size_t)dev]) != rocblas_status_success) {
    H.h[(size_t)dev] = nullptr;
    return nullptr;
  }
  rocblas_handle h = H.h[(size_t)dev];
  if (rocblas_set_stream(h, st) != rocblas_status_success) return nullptr;
  return h;
}

// K chunks of the products with a long contraction (V^H Q, V^H V: wb x N
// outputs, m rows): enough chunks that chunks x output tiles fill the device,
// chunks of at least 256 rows, partial products within 512 MiB.
inline int64_t ksplit(int64_t m, int64_t wb, int64_t N, size_t es) {
  const int64_t tiles = ((wb + 127) / 128) * ((N + 127) / 128);
  int64_t S = (768 + tiles - 1) / tiles;
  S = std::min<int64_t>(S, std::max<int64_t>(1, m / 256));
  const int64_t cap =
      std::max<int64_t>(1, (int64_t)((size_t(512) << 20) / ((size_t)wb * (size_t)N * es)));
  return std::max<int64_t>(1, std::min(S, cap));
}

// C (wb x N) = A^H B over m rows (A m x wb, lda; B m x N, ldb) as `chunks`
// K-chunk partial products in part, summed in a fixed order; rows of C
// scaled by tau when given.
template <typename E, typename S>
bool gemm_adj_splitk(rocblas_handle h, int64_t wb, int64_t N, int64_t m, const E* A, int64_t lda,
                     const E* B, int64_t ldb, int64_t chunks, E* part, const E* tau, E* C,
                     hipStream_t st) {
  const int64_t kc = (m + chunks - 1) / chunks;
  const int64_t full = m / kc, rem = m - full * kc;
  const auto A_ = Blas<E>::adj;
  const auto N_ = rocblas_operation_none;
  bool ok = true;
  if (full > 0)
    ok = Blas<E>::gemm_sb(h, A_, N_, wb, N, kc, S(1), A, lda, kc, B, ldb, kc, S(0), part, wb,
                          wb * N, full) == rocblas_status_success;
  if (ok && rem > 0)
    ok = Blas<E>::gemm(h, A_, N_, wb, N, rem, S(1), A + full * kc, lda, B + full * kc, ldb, S(0),
                       part + full * wb * N, wb) == rocblas_status_success;
  if (ok) {
    const int64_t total = wb * N;
    hipLaunchKernelGGL(k_sum_parts<E>, dim3((unsigned)std::min<int64_t>((total + 255) / 256, 8192)),
                       dim3(256), 0, st, part, full + (rem > 0 ? 1 : 0), total, tau, wb, C);
  }
  return ok;
}

}  // namespace ebt
