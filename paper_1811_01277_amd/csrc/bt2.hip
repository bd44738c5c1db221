// Band -> full back-transformation of eigenvectors (C ABI in
// include/elpa_bt2.h; Kus et al., Sec. 2): Q <- H_0 H_1 ... H_{n-nbw-1} Q
// with the first stage's reflectors H_c = I - tau_c v_c v_c^H, v_c on rows
// [c+nbw, n).
//
// Consecutive reflectors c0 .. c0+w-1 form one compact-WY product
//   H_c0 ... H_c0+w-1 = I - V T V^H
// (V the m x w block of vectors from row c0+nbw down, unit lead on the
// diagonal and zeros above it; T the upper triangular factor of the forward
// accumulation).  T is never formed: its inverse is diag(1/tau) +
// striu(V^H V), so
//   T W = (I + diag(tau) striu(V^H V))^{-1} (diag(tau) W),
// a row scaling and a unit upper triangular solve, with no division by tau
// (tau = 0, an identity reflector, is fine).  The blocks are applied last
// block first, each as
//   G = V^H V,  W = V^H Q[c0+nbw:, :],  W <- T W,  Q[c0+nbw:, :] -= V W,
// plain GEMMs and one triangular solve on the matrix cores through rocBLAS;
// packing V (explicit zeros and unit lead, so the vectors may share storage
// with anything above them), forming the unit triangle and scaling W are this
// file's kernels.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <algorithm>
#include <cstdint>
#include <mutex>
#include <vector>

#include "../../include/elpa_bt2.h"
#include "../../include/elpa_hh.h"

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

// Vp (m x wb, column major, ld m): column i = v_{c0+i} from row c0+nbw down,
// zero above row i, one at row i.
template <typename E>
__global__ __launch_bounds__(256) void k_pack(const E* __restrict__ V, int64_t ldv, int64_t nbw,
                                              int64_t c0, int64_t m, E* __restrict__ Vp) {
  const int64_t i = blockIdx.y;
  const int64_t c = c0 + i;
  E* __restrict__ dst = Vp + i * m;
  const E* __restrict__ src = V + c * ldv + c0 + nbw;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m;
       r += (int64_t)gridDim.x * blockDim.x) {
    E v;
    if (r < i)
      v = Num<E>::zero();
    else if (r == i)
      v = Num<E>::one();
    else
      v = src[r];
    dst[r] = v;
  }
}

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
  static rocblas_status trsm_unit_upper(rocblas_handle h, int64_t m, int64_t n, const double* A,
                                        int64_t lda, double* B, int64_t ldb) {
    const double one = 1.0;
    return rocblas_dtrsm_64(h, rocblas_side_left, rocblas_fill_upper, rocblas_operation_none,
                            rocblas_diagonal_unit, m, n, &one, A, lda, B, ldb);
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
  static rocblas_status trsm_unit_upper(rocblas_handle h, int64_t m, int64_t n, const float* A,
                                        int64_t lda, float* B, int64_t ldb) {
    const float one = 1.0f;
    return rocblas_strsm_64(h, rocblas_side_left, rocblas_fill_upper, rocblas_operation_none,
                            rocblas_diagonal_unit, m, n, &one, A, lda, B, ldb);
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
  static rocblas_status trsm_unit_upper(rocblas_handle h, int64_t m, int64_t n, const zc* A,
                                        int64_t lda, zc* B, int64_t ldb) {
    const rocblas_double_complex one{1.0, 0.0};
    return rocblas_ztrsm_64(h, rocblas_side_left, rocblas_fill_upper, rocblas_operation_none,
                            rocblas_diagonal_unit, m, n, &one, (const rocblas_double_complex*)A,
                            lda, (rocblas_double_complex*)B, ldb);
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

int64_t default_block(int32_t dtype) { return dtype == ELPA_C64 ? 192 : 384; }

// K chunks of the products with a long contraction (V^H Q, V^H V: wb x N
// outputs, m rows): enough chunks that chunks x output tiles fill the device,
// chunks of at least 256 rows, partial products within 512 MiB.
int64_t ksplit(int64_t m, int64_t wb, int64_t N, size_t es) {
  const int64_t tiles = ((wb + 127) / 128) * ((N + 127) / 128);
  int64_t S = (768 + tiles - 1) / tiles;
  S = std::min<int64_t>(S, std::max<int64_t>(1, m / 256));
  const int64_t cap =
      std::max<int64_t>(1, (int64_t)((size_t(512) << 20) / ((size_t)wb * (size_t)N * es)));
  return std::max<int64_t>(1, std::min(S, cap));
}

struct Layout {
  int64_t N = 0, w = 0, mmax = 0, nev = 0;
  size_t vp = 0, g = 0, t = 0, wbuf = 0, part = 0, total = 0;
  Layout(int64_t n, int64_t nev_, int64_t nbw, int64_t block, size_t es) {
    N = n > nbw ? n - nbw : 0;
    w = std::max<int64_t>(1, std::min<int64_t>(block, std::max<int64_t>(N, 1)));
    mmax = N;  // the first block's rows
    nev = nev_;
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    vp = al((size_t)mmax * w * es);
    g = al((size_t)w * w * es);
    t = al((size_t)w * w * es);
    wbuf = al((size_t)w * nev * es);
    // the largest set of partial products over all blocks
    size_t pe = 0;
    for (int64_t c0 = 0; c0 < N; c0 += w) {
      const int64_t wb = std::min<int64_t>(w, N - c0), m = N - c0;
      pe = std::max(pe, (size_t)ksplit(m, wb, nev, es) * wb * nev);
      pe = std::max(pe, (size_t)ksplit(m, wb, wb, es) * wb * wb);
    }
    part = al(pe * es);
    total = vp + g + t + wbuf + part;
  }
};

size_t elem_size(int32_t dtype) {
  switch (dtype) {
    case ELPA_R64: return 8;
    case ELPA_R32: return 4;
    case ELPA_C64: return 16;
    default: return 0;
  }
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

template <typename E, typename S>
int run(int64_t n, int64_t nev, int64_t nbw, const E* V, int64_t ldv, const E* tau, E* Q,
        int64_t ldq, hipStream_t st, int64_t block) {
  const Layout L(n, nev, nbw, block, sizeof(E));
  char* ws = nullptr;
  if (hipMallocAsync((void**)&ws, L.total, st) != hipSuccess) return ELPA_ERR_NOMEM;
  E* Vp = (E*)ws;
  E* G = (E*)(ws + L.vp);
  E* M = (E*)(ws + L.vp + L.g);
  E* W = (E*)(ws + L.vp + L.g + L.t);
  E* part = (E*)(ws + L.vp + L.g + L.t + L.wbuf);
  int dev = 0;
  (void)hipGetDevice(&dev);
  Handles& H = Handles::get();
  int rc = ELPA_OK;
  {
    std::lock_guard<std::mutex> lock(H.mu);
    if ((size_t)dev >= H.h.size()) H.h.resize((size_t)dev + 1, nullptr);
    if (!H.h[(size_t)dev] && rocblas_create_handle(&H.h[(size_t)dev]) != rocblas_status_success) {
      H.h[(size_t)dev] = nullptr;
      rc = ELPA_ERR_DEVICE;
    }
    rocblas_handle h = H.h[(size_t)dev];
    if (rc == ELPA_OK && rocblas_set_stream(h, st) != rocblas_status_success) rc = ELPA_ERR_DEVICE;
    const int64_t nblk = (L.N + L.w - 1) / L.w;
    for (int64_t b = nblk - 1; rc == ELPA_OK && b >= 0; --b) {
      const int64_t c0 = b * L.w;
      const int64_t wb = std::min<int64_t>(L.w, L.N - c0);
      const int64_t m = L.N - c0;  // rows c0+nbw .. n-1
      const unsigned gx = (unsigned)std::min<int64_t>((m + 255) / 256, 1024);
      hipLaunchKernelGGL(k_pack<E>, dim3(gx, (unsigned)wb), dim3(256), 0, st, V, ldv, nbw, c0, m,
                         Vp);
      E* Qs = Q + c0 + nbw;
      const auto N_ = rocblas_operation_none;
      // G = V^H V, then M = I + diag(tau) striu(G)
      bool ok = gemm_adj_splitk<E, S>(h, wb, wb, m, Vp, m, Vp, m,
                                      ksplit(m, wb, wb, sizeof(E)), part, nullptr, G, st);
      if (ok)
        hipLaunchKernelGGL(k_unit_tri<E>, dim3((unsigned)((wb * wb + 255) / 256)), dim3(256), 0,
                           st, G, tau + c0, wb, M);
      // W = diag(tau) V^H Q[c0+nbw:, :], then W <- M^{-1} W (= T V^H Q)
      ok = ok && gemm_adj_splitk<E, S>(h, wb, nev, m, Vp, m, Qs, ldq,
                                       ksplit(m, wb, nev, sizeof(E)), part, tau + c0, W, st);
      ok = ok && Blas<E>::trsm_unit_upper(h, wb, nev, M, wb, W, wb) == rocblas_status_success;
      ok = ok && Blas<E>::gemm(h, N_, N_, m, nev, wb, S(-1), Vp, m, W, wb, S(1), Qs, ldq) ==
                     rocblas_status_success;
      if (!ok || hipGetLastError() != hipSuccess) rc = ELPA_ERR_DEVICE;
    }
  }
  const hipError_t e2 = hipFreeAsync(ws, st);
  if (rc == ELPA_OK && e2 != hipSuccess) rc = ELPA_ERR_DEVICE;
  return rc;
}

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

}  // namespace ebt

extern "C" {

int64_t elpa_bt2_workspace_bytes(int64_t n, int64_t nev, int64_t nbw, int32_t dtype,
                                 int64_t block) {
  const size_t es = ebt::elem_size(dtype);
  if (n < 0 || nev < 0 || nbw < 1 || es == 0 || block < 0 || block > 512) return -1;
  if (n <= nbw || nev == 0) return 0;
  const ebt::Layout L(n, nev, nbw, block ? block : ebt::default_block(dtype), es);
  return (int64_t)L.total;
}

int elpa_bt2_trafo(int64_t n, int64_t nev, int64_t nbw, const void* V, int64_t ldv,
                   const void* tau, void* Q, int64_t ldq, int32_t dtype, void* stream,
                   int64_t block) {
  const size_t es = ebt::elem_size(dtype);
  if (es == 0) return ELPA_ERR_DTYPE;
  if (n < 0 || nev < 0 || nbw < 1 || block < 0 || block > 512) return ELPA_ERR_ARG;
  if (n <= nbw || nev == 0) return ELPA_OK;
  if (ldq < n || ldv < n || !V || !tau || !Q) return ELPA_ERR_ARG;
  if (!ebt::aligned(V, es) || !ebt::aligned(tau, es) || !ebt::aligned(Q, es))
    return ELPA_ERR_ALIGN;
  const int64_t b = block ? block : ebt::default_block(dtype);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  switch (dtype) {
    case ELPA_R64:
      return ebt::run<double, double>(n, nev, nbw, (const double*)V, ldv, (const double*)tau,
                                      (double*)Q, ldq, st, b);
    case ELPA_R32:
      return ebt::run<float, float>(n, nev, nbw, (const float*)V, ldv, (const float*)tau,
                                    (float*)Q, ldq, st, b);
    default:
      return ebt::run<ebt::zc, double>(n, nev, nbw, (const ebt::zc*)V, ldv,
                                       (const ebt::zc*)tau, (ebt::zc*)Q, ldq, st, b);
  }
}

}  // extern "C"
