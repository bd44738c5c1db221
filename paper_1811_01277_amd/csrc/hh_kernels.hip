// HIP kernels (gfx950) of the tridiagonal->band eigenvector back-transformation
//
//     Q <- H(0,0) H(0,1) ... H(n-2, J-1) Q,      H(s,j) = I - tau v v^H,
//
// the two-stage solver's first back-transformation (Kus et al., Sec. 2; the
// compute-heavy part singled out in Sec. 3.1).
//
// Mapping: one wave64 per stripe of 64 columns of Q, one lane per column.
// Columns never interact, so a lane owns its column for the whole call and
// no cross-lane communication is needed.  Reflector values are the same for
// every lane: they are read through the scalar unit (s_load into SGPRs) and
// enter the FMAs as the scalar operand.
//
// Order.  Sweeps are processed in blocks of K consecutive sweeps
// [s0, s0+K-1], blocks from the top (largest s) down.  Inside a block the
// chase steps run j = 0, 1, ..., and inside a step the sweeps run s0+K-1 down
// to s0.  Two reflectors (a, j) and (c, j') with a > c either do not share a
// row or are applied in the strict reverse generation order (if j < j' the
// rows of (a, j) end above those of (c, j') only when a - c >= b*(j'-j-1)+1,
// and a > c is already required), so the result equals strict reverse order
// up to rounding of the dot products.
//
// Window.  The K reflectors of step j of a block touch rows
// [s0+1+j*NB, s0+K-1+j*NB+NB], i.e. W = NB+K-1 rows; consecutive steps
// overlap in K-1 rows.  The stripe kernel keeps those W rows of its column in
// VGPRs, streams NB rows in and NB finished rows out per step, and applies
// K reflectors (2*NB*K FMAs per lane) per NB rows moved.
#include "hh_common.h"

namespace ehh {

// ---------------------------------------------------------------------------
// Reference kernel: any nbw, one reflector at a time in strict reverse
// generation order, the column kept in global memory.
// ---------------------------------------------------------------------------
template <typename E>
__global__ __launch_bounds__(64) void k_ref(const E* __restrict__ hh, const E* __restrict__ tau,
                                            E* __restrict__ Q, int64_t ldq, int64_t n,
                                            int64_t nev, int64_t nb) {
  using O = Ops<E>;
  const int64_t col = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (col >= nev) return;
  E* __restrict__ q = Q + col * ldq;
  const int64_t ctot = csum(n - 1, nb);
  for (int64_t s = n - 2; s >= 0; --s) {
    const int64_t off = ctot - csum(n - 1 - s, nb);
    const int64_t J = (n - 1 - s + nb - 1) / nb;
    for (int64_t j = J - 1; j >= 0; --j) {
      const int64_t slot = off + j;
      const int64_t r = s + 1 + j * nb;
      const int64_t L = (nb < n - r) ? nb : n - r;
      const E* __restrict__ v = hh + slot * nb;
      E acc = O::zero();
      for (int64_t i = 0; i < L; ++i) O::dot(acc, v[i], q[r + i]);
      const E w = O::scale(acc, tau[slot]);
      for (int64_t i = 0; i < L; ++i) O::axpy(q[r + i], v[i], w);
    }
  }
}

// ---------------------------------------------------------------------------
// Stripe kernel: register window of W = NB+K-1 rows per lane, K sweeps fused.
// ---------------------------------------------------------------------------
template <typename E, int NB, int K>
__global__ __launch_bounds__(64, 1) void k_stripe(const E* __restrict__ hh,
                                                  const E* __restrict__ tau,
                                                  E* __restrict__ Q, int64_t ldq, int64_t n,
                                                  int64_t nev) {
  using O = Ops<E>;
  constexpr int W = NB + K - 1;
  const int64_t col = (int64_t)blockIdx.x * 64 + threadIdx.x;
  const bool act = col < nev;
  E* __restrict__ q = Q + (act ? col : 0) * ldq;
  const int64_t nblk = (n - 1 + K - 1) / K;
  const int64_t ctot = csum(n - 1, NB);
  E x[W];
  for (int64_t m = nblk - 1; m >= 0; --m) {
    const int64_t s0 = m * K;
    const int64_t s1 = (s0 + K - 1 < n - 2) ? s0 + K - 1 : n - 2;
    const int64_t base = s0 + 1;
    const int64_t J0 = (n - 1 - s0 + NB - 1) / NB;
#pragma unroll
    for (int i = 0; i < W; ++i) {
      const int64_t r = base + i;
      x[i] = (act && r < n) ? q[r] : O::zero();
    }
    for (int64_t j = 0; j < J0; ++j) {
      const int64_t row0 = base + j * NB;
      if (j > 0) {
#pragma unroll
        for (int i = 0; i < K - 1; ++i) x[i] = x[i + NB];
#pragma unroll
        for (int i = K - 1; i < W; ++i) {
          const int64_t r = row0 + i;
          x[i] = (act && r < n) ? q[r] : O::zero();
        }
      }
#pragma unroll
      for (int o = K - 1; o >= 0; --o) {
        const int64_t s = s0 + o;
        if (s > s1 || s + 1 + j * NB >= n) continue;
        const int64_t slot = ctot - csum(n - 1 - s, NB) + j;
        const E* __restrict__ v = hh + slot * NB;
        E a0 = O::zero(), a1 = O::zero(), a2 = O::zero(), a3 = O::zero();
#pragma unroll
        for (int i = 0; i < NB; i += 4) {
          O::dot(a0, v[i + 0], x[o + i + 0]);
          O::dot(a1, v[i + 1], x[o + i + 1]);
          O::dot(a2, v[i + 2], x[o + i + 2]);
          O::dot(a3, v[i + 3], x[o + i + 3]);
        }
        const E w = O::scale(O::add(O::add(a0, a1), O::add(a2, a3)), tau[slot]);
#pragma unroll
        for (int i = 0; i < NB; ++i) O::axpy(x[o + i], v[i], w);
      }
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const int64_t r = row0 + i;
        if (act && r < n) q[r] = x[i];
      }
    }
    const int64_t rowl = base + (J0 - 1) * NB;
#pragma unroll
    for (int i = NB; i < W; ++i) {
      const int64_t r = rowl + i;
      if (act && r < n) q[r] = x[i];
    }
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename E>
hipError_t launch_ref(const void* hh, const void* tau, void* Q, int64_t ldq, int64_t n,
                      int64_t nev, int64_t nb, hipStream_t st) {
  const dim3 grid((unsigned)((nev + 63) / 64)), block(64);
  hipLaunchKernelGGL(k_ref<E>, grid, block, 0, st, (const E*)hh, (const E*)tau, (E*)Q, ldq, n,
                     nev, nb);
  return hipGetLastError();
}

template <typename E, int NB, int K>
hipError_t launch_stripe(const void* hh, const void* tau, void* Q, int64_t ldq, int64_t n,
                         int64_t nev, hipStream_t st) {
  const dim3 grid((unsigned)((nev + 63) / 64)), block(64);
  hipLaunchKernelGGL((k_stripe<E, NB, K>), grid, block, 0, st, (const E*)hh, (const E*)tau,
                     (E*)Q, ldq, n, nev);
  return hipGetLastError();
}

}  // namespace ehh

// Table of compiled stripe variants, consumed by the C ABI.
#include "hh_dispatch.h"

namespace ehh {

#define EHH_STRIPE(E, DT, NB, K) {DT, NB, K, &launch_stripe<E, NB, K>}

const StripeEntry* stripe_table(int* size) {
  static const StripeEntry table[] = {
      EHH_STRIPE(double, 0, 32, 1),  EHH_STRIPE(double, 0, 32, 2),  EHH_STRIPE(double, 0, 32, 4),
      EHH_STRIPE(double, 0, 32, 6),  EHH_STRIPE(double, 0, 32, 8),  EHH_STRIPE(double, 0, 32, 16),
      EHH_STRIPE(double, 0, 32, 32), EHH_STRIPE(double, 0, 64, 1),  EHH_STRIPE(double, 0, 64, 2),
      EHH_STRIPE(double, 0, 64, 4),  EHH_STRIPE(double, 0, 64, 6),  EHH_STRIPE(double, 0, 64, 8),
      EHH_STRIPE(double, 0, 64, 16),
      EHH_STRIPE(float, 1, 32, 1),   EHH_STRIPE(float, 1, 32, 4),   EHH_STRIPE(float, 1, 32, 16),
      EHH_STRIPE(float, 1, 32, 32),  EHH_STRIPE(float, 1, 64, 1),   EHH_STRIPE(float, 1, 64, 4),
      EHH_STRIPE(float, 1, 64, 16),
      EHH_STRIPE(z64, 2, 32, 1),     EHH_STRIPE(z64, 2, 32, 2),     EHH_STRIPE(z64, 2, 32, 4),
      EHH_STRIPE(z64, 2, 64, 2),
  };
  *size = (int)(sizeof(table) / sizeof(table[0]));
  return table;
}

RefLaunch ref_launcher(int dtype) {
  switch (dtype) {
    case 0: return &launch_ref<double>;
    case 1: return &launch_ref<float>;
    case 2: return &launch_ref<z64>;
    default: return nullptr;
  }
}

}  // namespace ehh
