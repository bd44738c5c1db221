// Generalized Hermitian-definite eigenproblem (C ABI in include/elpa_gen.h;
// Kus et al., Sec. 2 and Sec. 4 "Generalized EVP problem").
//
// Cholesky B = L L^H, blocked right-looking over panels of nb = 64 columns:
//   the diagonal block is factored in LDS by one workgroup with the column
//   recurrence (a pivot that is not positive is recorded in *info);
//   the panel below:     B21 <- B21 L11^{-H}  (triangular solve);
//   the trailing matrix: B22 -= B21 B21^H     (Hermitian rank-nb update of the
//   lower triangle).
// The inverse L^{-1} is formed by rocBLAS trtri in a workspace and copied into
// B's lower triangle, zeros above.  The two transformations are triangular
// multiplications (rocBLAS trmm, out of place through a workspace):
//   A <- Linv A Linv^H (then averaged with its adjoint so that it is exactly
//   Hermitian), Q <- Linv^H Q.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <mutex>

#include "../../include/elpa_gen.h"
#include "../../include/elpa_hh.h"
#include "wy_blas.h"

namespace egen {

using ebt::zc;

constexpr int64_t kNb = 64;  // Cholesky panel width (the diagonal block fits in LDS)

__device__ __forceinline__ double re(double a) { return a; }
__device__ __forceinline__ double re(zc a) { return a.re; }
__device__ __forceinline__ double conj_(double a) { return a; }
__device__ __forceinline__ zc conj_(zc a) { return zc{a.re, -a.im}; }
__device__ __forceinline__ double div_re(double a, double l) { return a / l; }
__device__ __forceinline__ zc div_re(zc a, double l) { return zc{a.re / l, a.im / l}; }
__device__ __forceinline__ double fms(double c, double a, double b) { return c - a * b; }
__device__ __forceinline__ zc fms(zc c, zc a, zc b) {
  return zc{c.re - (a.re * b.re - a.im * b.im), c.im - (a.re * b.im + a.im * b.re)};
}
__device__ __forceinline__ double avg_adj(double a, double b) { return 0.5 * (a + b); }
// (a + conj(b)) / 2
__device__ __forceinline__ zc avg_adj(zc a, zc b) {
  return zc{0.5 * (a.re + b.re), 0.5 * (a.im - b.im)};
}
template <typename E>
__device__ __forceinline__ E from_re(double x);
template <>
__device__ __forceinline__ double from_re<double>(double x) { return x; }
template <>
__device__ __forceinline__ zc from_re<zc>(double x) { return zc{x, 0.0}; }

__global__ void k_clear_info(int32_t* info) { *info = 0; }

// Factor the diagonal block B[j0:j0+jb, j0:j0+jb] (jb <= kNb) in place, lower
// triangle, one workgroup, column by column on a copy in LDS; skipped once
// *info is set.
template <typename E>
__global__ __launch_bounds__(256) void k_potrf_diag(E* __restrict__ B, int64_t ldb, int64_t j0,
                                                    int64_t jb, int32_t* __restrict__ info) {
  __shared__ E sh[kNb][kNb + 1];  // sh[col][row]
  __shared__ int failed;
  const int tid = threadIdx.x;
  if (tid == 0) failed = *info;
  E* const blk = B + j0 * ldb + j0;
  for (int64_t e = tid; e < jb * jb; e += blockDim.x) {
    const int64_t i = e % jb, j = e / jb;
    if (i >= j) sh[j][i] = blk[j * ldb + i];
  }
  __syncthreads();
  if (failed) return;
  int64_t k = 0;
  for (; k < jb; ++k) {
    const double d = re(sh[k][k]);
    if (!(d > 0.0)) {  // uniform: every thread read the same entry
      if (tid == 0) *info = (int32_t)(j0 + k + 1);
      break;
    }
    const double l = sqrt(d);
    for (int64_t i = k + 1 + tid; i < jb; i += blockDim.x) sh[k][i] = div_re(sh[k][i], l);
    __syncthreads();
    if (tid == 0) sh[k][k] = from_re<E>(l);
    const int64_t r = jb - k - 1;
    for (int64_t e = tid; e < r * r; e += blockDim.x) {
      const int64_t i = e % r, j = e / r;
      if (i >= j) sh[k + 1 + j][k + 1 + i] = fms(sh[k + 1 + j][k + 1 + i], sh[k][k + 1 + i],
                                                 conj_(sh[k][k + 1 + j]));
    }
    __syncthreads();
  }
  if (k < jb) return;  // failed: B's contents are unspecified
  for (int64_t e = tid; e < jb * jb; e += blockDim.x) {
    const int64_t i = e % jb, j = e / jb;
    if (i >= j) blk[j * ldb + i] = sh[j][i];
  }
}

// B[i, j] = W[i, j] for i >= j, 0 above (n x n; W with ld n).
template <typename E>
__global__ __launch_bounds__(256) void k_copy_lower(const E* __restrict__ W, int64_t n,
                                                    E* __restrict__ B, int64_t ldb) {
  for (int64_t j = blockIdx.y; j < n; j += gridDim.y)
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
      B[j * ldb + i] = i >= j ? W[j * n + i] : from_re<E>(0.0);
}

// A <- (A + A^H) / 2 by 32 x 32 tile pairs (lower tile L, its mirror U):
// L[r][c] <- (L[r][c] + conj(U[c][r])) / 2 and U[r][c] <- (U[r][c] +
// conj(L[c][r])) / 2; a diagonal tile is its own mirror.
template <typename E>
__global__ __launch_bounds__(256) void k_hermitize(E* __restrict__ A, int64_t lda, int64_t n) {
  const int64_t bi = blockIdx.x, bj = blockIdx.y;
  if (bj > bi) return;
  __shared__ E sl[32][33];
  __shared__ E su[32][33];
  const int tr = threadIdx.x & 31, tc0 = threadIdx.x >> 5;  // 8 column lanes
  for (int c = tc0; c < 32; c += 8) {
    const int64_t i = bi * 32 + tr, j = bj * 32 + c;
    if (i < n && j < n) sl[tr][c] = A[j * lda + i];
    const int64_t i2 = bj * 32 + tr, j2 = bi * 32 + c;
    if (i2 < n && j2 < n) su[tr][c] = A[j2 * lda + i2];
  }
  __syncthreads();
  for (int c = tc0; c < 32; c += 8) {
    const int64_t i = bi * 32 + tr, j = bj * 32 + c;
    if (i < n && j < n) A[j * lda + i] = avg_adj(sl[tr][c], su[c][tr]);
    if (bi != bj) {
      const int64_t i2 = bj * 32 + tr, j2 = bi * 32 + c;
      if (i2 < n && j2 < n) A[j2 * lda + i2] = avg_adj(su[tr][c], sl[c][tr]);
    }
  }
}

template <typename E>
struct Lapack;
template <>
struct Lapack<double> {
  static rocblas_status trsm_rlc(rocblas_handle h, int64_t m, int64_t n, const double* A,
                                 int64_t lda, double* B, int64_t ldb) {
    const double one = 1.0;
    return rocblas_dtrsm_64(h, rocblas_side_right, rocblas_fill_lower,
                            rocblas_operation_transpose, rocblas_diagonal_non_unit, m, n, &one, A,
                            lda, B, ldb);
  }
  static rocblas_status herk_ln(rocblas_handle h, int64_t n, int64_t k, const double* A,
                                int64_t lda, double* C, int64_t ldc) {
    const double a = -1.0, b = 1.0;
    return rocblas_dsyrk_64(h, rocblas_fill_lower, rocblas_operation_none, n, k, &a, A, lda, &b, C,
                            ldc);
  }
  static rocblas_status trtri_l(rocblas_handle h, int64_t n, const double* A, int64_t lda,
                                double* W, int64_t ldw) {
    return rocblas_dtrtri(h, rocblas_fill_lower, rocblas_diagonal_non_unit, (rocblas_int)n, A,
                          (rocblas_int)lda, W, (rocblas_int)ldw);
  }
  static rocblas_status trmm_l(rocblas_handle h, rocblas_side side, rocblas_operation op,
                               int64_t m, int64_t n, const double* L, int64_t ldl,
                               const double* B, int64_t ldb, double* C, int64_t ldc) {
    const double one = 1.0;
    return rocblas_dtrmm_64(h, side, rocblas_fill_lower, op, rocblas_diagonal_non_unit, m, n, &one,
                            L, ldl, B, ldb, C, ldc);
  }
  static constexpr rocblas_operation adj = rocblas_operation_transpose;
};
template <>
struct Lapack<zc> {
  using Z = rocblas_double_complex;
  static rocblas_status trsm_rlc(rocblas_handle h, int64_t m, int64_t n, const zc* A, int64_t lda,
                                 zc* B, int64_t ldb) {
    const Z one{1.0, 0.0};
    return rocblas_ztrsm_64(h, rocblas_side_right, rocblas_fill_lower,
                            rocblas_operation_conjugate_transpose, rocblas_diagonal_non_unit, m, n,
                            &one, (const Z*)A, lda, (Z*)B, ldb);
  }
  static rocblas_status herk_ln(rocblas_handle h, int64_t n, int64_t k, const zc* A, int64_t lda,
                                zc* C, int64_t ldc) {
    const double a = -1.0, b = 1.0;
    return rocblas_zherk_64(h, rocblas_fill_lower, rocblas_operation_none, n, k, &a, (const Z*)A,
                            lda, &b, (Z*)C, ldc);
  }
  static rocblas_status trtri_l(rocblas_handle h, int64_t n, const zc* A, int64_t lda, zc* W,
                                int64_t ldw) {
    return rocblas_ztrtri(h, rocblas_fill_lower, rocblas_diagonal_non_unit, (rocblas_int)n,
                          (const Z*)A, (rocblas_int)lda, (Z*)W, (rocblas_int)ldw);
  }
  static rocblas_status trmm_l(rocblas_handle h, rocblas_side side, rocblas_operation op,
                               int64_t m, int64_t n, const zc* L, int64_t ldl, const zc* B,
                               int64_t ldb, zc* C, int64_t ldc) {
    const Z one{1.0, 0.0};
    return rocblas_ztrmm_64(h, side, rocblas_fill_lower, op, rocblas_diagonal_non_unit, m, n, &one,
                            (const Z*)L, ldl, (const Z*)B, ldb, (Z*)C, ldc);
  }
  static constexpr rocblas_operation adj = rocblas_operation_conjugate_transpose;
};

#define EGEN_OK(x) ((x) == rocblas_status_success)

template <typename E>
int cholesky_inverse(int64_t n, E* B, int64_t ldb, int32_t* info, hipStream_t st) {
  E* W = nullptr;
  if (hipMallocAsync((void**)&W, (size_t)n * n * sizeof(E), st) != hipSuccess)
    return ELPA_ERR_NOMEM;
  int rc = ELPA_OK;
  hipLaunchKernelGGL(k_clear_info, dim3(1), dim3(1), 0, st, info);
  {
    std::lock_guard<std::mutex> lock(ebt::Handles::get().mu);
    rocblas_handle h = ebt::handle_for(st);
    bool ok = h != nullptr;
    for (int64_t j0 = 0; ok && j0 < n; j0 += kNb) {
      const int64_t jb = std::min(kNb, n - j0), m = n - j0 - jb;
      hipLaunchKernelGGL(k_potrf_diag<E>, dim3(1), dim3(256), 0, st, B, ldb, j0, jb, info);
      if (m > 0) {
        E* L11 = B + j0 * ldb + j0;
        E* B21 = L11 + jb;
        E* B22 = B + (j0 + jb) * ldb + j0 + jb;
        ok = ok && EGEN_OK(Lapack<E>::trsm_rlc(h, m, jb, L11, ldb, B21, ldb));
        ok = ok && EGEN_OK(Lapack<E>::herk_ln(h, m, jb, B21, ldb, B22, ldb));
      }
    }
    ok = ok && EGEN_OK(Lapack<E>::trtri_l(h, n, B, ldb, W, n));
    if (ok)
      hipLaunchKernelGGL(k_copy_lower<E>, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 64),
                                               (unsigned)std::min<int64_t>(n, 65535)),
                         dim3(256), 0, st, (const E*)W, n, B, ldb);
    if (!ok || hipGetLastError() != hipSuccess) rc = ELPA_ERR_DEVICE;
  }
  const hipError_t e2 = hipFreeAsync(W, st);
  if (rc == ELPA_OK && e2 != hipSuccess) rc = ELPA_ERR_DEVICE;
  return rc;
}

template <typename E>
int to_standard(int64_t n, E* A, int64_t lda, const E* L, int64_t ldl, hipStream_t st) {
  E* W = nullptr;
  if (hipMallocAsync((void**)&W, (size_t)n * n * sizeof(E), st) != hipSuccess)
    return ELPA_ERR_NOMEM;
  int rc = ELPA_OK;
  {
    std::lock_guard<std::mutex> lock(ebt::Handles::get().mu);
    rocblas_handle h = ebt::handle_for(st);
    bool ok = h != nullptr;
    // W = Linv A, then A = W Linv^H
    ok = ok && EGEN_OK(Lapack<E>::trmm_l(h, rocblas_side_left, rocblas_operation_none, n, n, L,
                                         ldl, A, lda, W, n));
    ok = ok && EGEN_OK(Lapack<E>::trmm_l(h, rocblas_side_right, Lapack<E>::adj, n, n, L, ldl, W,
                                         n, A, lda));
    if (ok) {
      const unsigned nt = (unsigned)((n + 31) / 32);
      hipLaunchKernelGGL(k_hermitize<E>, dim3(nt, nt), dim3(256), 0, st, A, lda, n);
    }
    if (!ok || hipGetLastError() != hipSuccess) rc = ELPA_ERR_DEVICE;
  }
  const hipError_t e2 = hipFreeAsync(W, st);
  if (rc == ELPA_OK && e2 != hipSuccess) rc = ELPA_ERR_DEVICE;
  return rc;
}

template <typename E>
int back(int64_t n, int64_t nev, const E* L, int64_t ldl, E* Q, int64_t ldq, hipStream_t st) {
  E* W = nullptr;
  if (hipMallocAsync((void**)&W, (size_t)n * nev * sizeof(E), st) != hipSuccess)
    return ELPA_ERR_NOMEM;
  int rc = ELPA_OK;
  {
    std::lock_guard<std::mutex> lock(ebt::Handles::get().mu);
    rocblas_handle h = ebt::handle_for(st);
    bool ok = h != nullptr;
    ok = ok && EGEN_OK(Lapack<E>::trmm_l(h, rocblas_side_left, Lapack<E>::adj, n, nev, L, ldl, Q,
                                         ldq, W, n));
    ok = ok && hipMemcpy2DAsync(Q, (size_t)ldq * sizeof(E), W, (size_t)n * sizeof(E),
                                (size_t)n * sizeof(E), (size_t)nev, hipMemcpyDeviceToDevice,
                                st) == hipSuccess;
    if (!ok || hipGetLastError() != hipSuccess) rc = ELPA_ERR_DEVICE;
  }
  const hipError_t e2 = hipFreeAsync(W, st);
  if (rc == ELPA_OK && e2 != hipSuccess) rc = ELPA_ERR_DEVICE;
  return rc;
}

size_t elem(int32_t dtype) { return dtype == ELPA_R64 ? 8 : dtype == ELPA_C64 ? 16 : 0; }
bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

}  // namespace egen

extern "C" {

int elpa_cholesky_inverse(int64_t n, void* B, int64_t ldb, int32_t dtype, void* stream,
                          int32_t* info) {
  const size_t es = egen::elem(dtype);
  if (es == 0) return ELPA_ERR_DTYPE;
  if (n < 0 || n > INT_MAX || ldb < std::max<int64_t>(n, 1) || ldb > INT_MAX) return ELPA_ERR_ARG;
  if (n == 0) return ELPA_OK;
  if (!B || !info) return ELPA_ERR_ARG;
  if (!egen::aligned(B, es) || !egen::aligned(info, 4)) return ELPA_ERR_ALIGN;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (dtype == ELPA_R64) return egen::cholesky_inverse<double>(n, (double*)B, ldb, info, st);
  return egen::cholesky_inverse<ebt::zc>(n, (ebt::zc*)B, ldb, info, st);
}

int elpa_generalized_to_standard(int64_t n, void* A, int64_t lda, const void* Linv, int64_t ldl,
                                 int32_t dtype, void* stream) {
  const size_t es = egen::elem(dtype);
  if (es == 0) return ELPA_ERR_DTYPE;
  if (n < 0 || lda < std::max<int64_t>(n, 1) || ldl < std::max<int64_t>(n, 1))
    return ELPA_ERR_ARG;
  if (n == 0) return ELPA_OK;
  if (!A || !Linv) return ELPA_ERR_ARG;
  if (!egen::aligned(A, es) || !egen::aligned(Linv, es)) return ELPA_ERR_ALIGN;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (dtype == ELPA_R64)
    return egen::to_standard<double>(n, (double*)A, lda, (const double*)Linv, ldl, st);
  return egen::to_standard<ebt::zc>(n, (ebt::zc*)A, lda, (const ebt::zc*)Linv, ldl, st);
}

int elpa_generalized_back(int64_t n, int64_t nev, const void* Linv, int64_t ldl, void* Q,
                          int64_t ldq, int32_t dtype, void* stream) {
  const size_t es = egen::elem(dtype);
  if (es == 0) return ELPA_ERR_DTYPE;
  if (n < 0 || nev < 0 || ldl < std::max<int64_t>(n, 1) || ldq < std::max<int64_t>(n, 1))
    return ELPA_ERR_ARG;
  if (n == 0 || nev == 0) return ELPA_OK;
  if (!Linv || !Q) return ELPA_ERR_ARG;
  if (!egen::aligned(Q, es) || !egen::aligned(Linv, es)) return ELPA_ERR_ALIGN;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (dtype == ELPA_R64)
    return egen::back<double>(n, nev, (const double*)Linv, ldl, (double*)Q, ldq, st);
  return egen::back<ebt::zc>(n, nev, (const ebt::zc*)Linv, ldl, (ebt::zc*)Q, ldq, st);
}

}  // extern "C"
