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
#include "wy_blas.h"

namespace ebt {

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

int64_t default_block(int32_t dtype) { return dtype == ELPA_C64 ? 192 : 384; }

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
  int rc = ELPA_OK;
  {
    std::lock_guard<std::mutex> lock(Handles::get().mu);
    rocblas_handle h = handle_for(st);
    if (!h) rc = ELPA_ERR_DEVICE;
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
      ok = ok && Blas<E>::trsm(h, rocblas_side_left, rocblas_operation_none, wb, nev, M, wb, W,
                               wb) == rocblas_status_success;
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
