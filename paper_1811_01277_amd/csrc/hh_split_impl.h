// Split-window stripe kernel (real and complex fp64) of the tridiagonal->band eigenvector
// back-transformation  Q <- H(0,0) H(0,1) ... H(n-2, J-1) Q  (Kus et al.,
// Sec. 2 and Sec. 3.1).
//
// Same block/step structure and diagonal launch schedule as the one-lane
// stripe kernel (blocks of K sweeps slide a window of W = NB+K-1 rows down a
// stripe, one chase step at a time; launch t runs every tile (stripe c, block
// m, group q of S steps) with (M-1-m)+q = t), with three differences:
//
// 1. Two lanes per column.  A wave covers 32 columns; lane l = 32h + c holds
//    the window rows of parity h of column c.  A lane keeps R = (NB+K)/2
//    registers instead of NB+K-1, so K (the reuse of every loaded row, the
//    kernel's arithmetic intensity is K/4 flop per byte) can be about twice
//    as large for the same register budget, and the unrolled step body is half
//    as long per reflector (it has to stay inside the instruction cache).
//    Reflector o of a step (window rows o..o+NB-1) meets, in each lane half,
//    the registers p = o/2 .. o/2+NB/2-1 (even o) or (o-1)/2 .. (o-1)/2+NB/2
//    (odd o: one more register, whose reflector value is zero in one half).
//    The two halves' partial dot products are combined with a lane swap
//    across the halves (v_permlane32_swap), identically in both halves.
//    Real reflectors are applied in pairs (odd o, then o-1), which start on
//    the same register: two dot products in one pass, a 2x2 triangular
//    correction with the pair coupling, and one update pass, as the paper's
//    CPU kernels fuse two or more reflectors (Sec. 3.1).
// 2. Packed reflectors.  A pre-pass writes, for every (block m, step j,
//    offset o), the reflector (m*K+o, j) in the order the lanes consume it:
//    per lane half HN+1 values (index 2t+h-(o&1) of v, zero outside [0, L)),
//    tau in the first half's spare slot, for real records of even o the pair
//    coupling v(o).v(o+1) in the second half's, zeros for reflectors that do
//    not exist.  The step body then needs no slot arithmetic and no branches.
// 3. Stripes are 32 columns wide; a stripe row pair (rows 2p, 2p+1) is one
//    contiguous 512-byte access of the wave.
//
// The extra window row (W is odd, the register file holds W+1 rows) is
// loaded but never written; it lies one row short of the next block's tile
// in the same launch.
#pragma once

#include "hh_common.h"
#include "hh_dispatch.h"
#include "hh_dpp.h"
#include "hh_layout.h"
#include "hh_sched.h"

namespace ehh {

template <int NB, int K>
struct SplitGeom {
  static_assert(NB == 32 || NB == 64, "split kernel supports NB = 32, 64");
  static_assert(K >= 2 && K % 2 == 0, "split kernel needs an even K");
  static constexpr int HN = NB / 2;       // window rows per lane half and reflector
  static constexpr int NG = NB / 32;      // full 16-value segments per lane half
  static constexpr int HS = HN + 2;       // packed half: HN+1 values, then tau / zero
  static constexpr int RS = 2 * HS;       // packed reflector record
  static constexpr int R = (NB + K) / 2;  // registers per lane (W + 1 rows)
  static constexpr int64_t SW = 32;       // columns per stripe
};

// Packed record of reflector (s0+o, j), o = 0..K-1, written by one block.
// The records of every block's existing steps are stored back to back; block
// m's first step record is Bt[m] = block_base(m), written here (step 0) for
// the apply kernels, which read it once per tile.
template <typename E, int NB, int K>
__device__ __forceinline__ void pack_group(const E* __restrict__ hh, const E* __restrict__ tau,
                                           int64_t n, int64_t m, int64_t j,
                                           E* __restrict__ P, int64_t* __restrict__ Bt) {
  using Gm = SplitGeom<NB, K>;
  const int64_t s0 = m * K;
  const int64_t J0 = block_steps(n, NB, K, m);
  if (j >= J0) return;  // no such step
  const int64_t ctot = csum(n - 1, NB);
  const int64_t mb = block_base(n, NB, K, m);
  if (j == 0 && threadIdx.x == 0) Bt[m] = mb;
  E* __restrict__ rec = P + ((mb + j) * K) * Gm::RS;
  for (int e = (int)threadIdx.x; e < K * Gm::RS; e += (int)blockDim.x) {
    const int o = e / Gm::RS, rem = e - o * Gm::RS;
    const int h = rem / Gm::HS, t = rem - h * Gm::HS;
    const int64_t s = s0 + o;
    const bool valid = (s <= n - 2) && (j < (n - 1 - s + NB - 1) / NB);
    E v{};
    if (valid) {
      const int64_t slot = ctot - csum(n - 1 - s, NB) + j;
      if (h == 0 && t == Gm::HS - 1) {
        v = tau[slot];
      } else {
        const int64_t r = s + 1 + j * NB;
        const int64_t L = (NB < n - r) ? NB : n - r;
        const int i = 2 * t + h - (o & 1);
        if (i >= 0 && i < L) v = hh[slot * NB + i];
      }
    }
    // real records: the second half's spare slot of an even offset holds the
    // pair coupling, written below
    if (std::is_floating_point<E>::value && h == 1 && t == Gm::HS - 1 && (o & 1) == 0) continue;
    rec[e] = v;
  }
  if constexpr (std::is_floating_point<E>::value) {
    // pair coupling c = vB.vA of B = offset o (even) and A = o+1 (vA starts one
    // window row below vB): one wave per pair, a fixed-order tree sum in fp64
    const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
    for (int o = 2 * wave; o < K; o += 2 * ((int)blockDim.x >> 6)) {
      const int64_t s = s0 + o, sa = s + 1;
      const bool vb = (s <= n - 2) && (j < (n - 1 - s + NB - 1) / NB);
      const bool va = o + 1 < K && (sa <= n - 2) && (j < (n - 1 - sa + NB - 1) / NB);
      double prod = 0.0;
      if (vb && va) {
        const int64_t rb = s + 1 + j * NB;
        const int64_t lb = (NB < n - rb) ? NB : n - rb;
        const int64_t la = (NB < n - rb - 1) ? NB : n - rb - 1;
        if (lane + 1 < lb && lane < la) {
          const int64_t slot_b = ctot - csum(n - 1 - s, NB) + j;
          const int64_t slot_a = ctot - csum(n - 1 - sa, NB) + j;
          prod = (double)hh[slot_b * NB + lane + 1] * (double)hh[slot_a * NB + lane];
        }
      }
#pragma unroll
      for (int w = 32; w >= 1; w >>= 1) prod += __shfl_xor(prod, w, 64);
      if (lane == 0) rec[o * Gm::RS + Gm::RS - 1] = (E)prod;
    }
  }
}

template <typename E, int NB, int K>
__global__ __launch_bounds__(256) void k_pack_split(const E* __restrict__ hh,
                                                    const E* __restrict__ tau, int64_t n,
                                                    int64_t Jmax, E* __restrict__ P,
                                                    int64_t* __restrict__ Bt) {
  const int64_t g = blockIdx.x;
  pack_group<E, NB, K>(hh, tau, n, g / Jmax, g % Jmax, P, Bt);
}

template <typename E, int NB, int K>
__global__ __launch_bounds__(256) void k_pack_split_b(const ProblemDesc* __restrict__ d,
                                                      int count) {
  const int b = (int)blockIdx.x;
  const ProblemDesc& D = d[find_by<ProblemDesc, &ProblemDesc::ptile0>(d, count, b)];
  const int64_t g = b - D.ptile0;
  pack_group<E, NB, K>((const E*)D.hh, (const E*)D.tau, D.n, g / D.Jmax, g % D.Jmax, (E*)D.P,
                       (int64_t*)D.Bt);
}

// Sum of a value over the two lane halves (lanes l and l^32), computed in the
// same order in both halves so that they agree bitwise.
__device__ __forceinline__ double half_pair_sum(double s) {
  const unsigned lo = (unsigned)__double2loint(s), hi = (unsigned)__double2hiint(s);
  const auto rl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto rh = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  // element 0: lower half's value in every lane; element 1: upper half's
  return __hiloint2double((int)rh[0], (int)rl[0]) + __hiloint2double((int)rh[1], (int)rl[1]);
}

__device__ __forceinline__ float half_pair_sum(float s) {
  const unsigned u = __float_as_uint(s);
  const auto r = __builtin_amdgcn_permlane32_swap(u, u, false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Reflector pairs (A = odd offset o, applied first; B = o-1): the two dot
// products wA = vA.x and wB = vB.x are taken together on the window as it is
// before A, and B's is corrected for A's update with the pair coupling
// c = vB.vA, stored by the packing pass in B's record:
//   nwA = -tauA wA,  nwB = -tauB (wB + c nwA),  x += vA nwA + vB nwB,
// which is (I - tauB vB vB^T)(I - tauA vA vA^T) x.  Both reflectors start on
// register o/2 of each lane half; one reduction across the halves serves the
// pair.
template <typename T>
struct SplitPair {
  T a0, a1, a2, ta, b0, b1, tb, c;
};

template <int NB, int K, int o, typename T>
__device__ __forceinline__ SplitPair<T> split_load_pair(const T* __restrict__ Pj, int voff,
                                                        int z) {
  using Gm = SplitGeom<NB, K>;
  static_assert((o & 1) == 1, "A is the odd offset of a pair");
  const T* __restrict__ ra = Pj + o * Gm::RS + z;
  const T* __restrict__ rb = ra - Gm::RS;
  SplitPair<T> s;
  s.a0 = ra[voff];
  s.a1 = (Gm::NG == 2) ? ra[voff + 16] : T(0);
  s.a2 = ra[voff + 16 * Gm::NG];
  s.ta = ra[Gm::HS - 1];
  s.b0 = rb[voff];
  s.b1 = (Gm::NG == 2) ? rb[voff + 16] : T(0);
  s.tb = rb[Gm::HS - 1];
  s.c = rb[Gm::RS - 1];
  return s;
}

// T = double or float (the same blocks on 64- or 32-bit values)
template <int NB, int K, int PD, typename T, int R>
__device__ __forceinline__ void step_split_pair(T (&x)[R], const T* __restrict__ Pj, int voff) {
  using Gm = SplitGeom<NB, K>;
  constexpr int NP = K / 2, HN = Gm::HN, NG = Gm::NG;
  static_assert(R == Gm::R, "window register count");
  static_assert(PD >= 1 && PD <= 3 && PD < NP, "pair prefetch distance 1..3");
  SplitPair<T> buf[PD];
  FwdFor<PD>::run([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    buf[i] = split_load_pair<NB, K, K - 1 - 2 * i>(Pj, voff, 0);
  });
  RevFor<NP>::run([&](auto pc) {
    constexpr int pi = decltype(pc)::value;
    constexpr int p0 = pi;  // (2 pi + 1) >> 1
    const SplitPair<T> c0 = buf[0];
    T aA0 = T(0), aA1 = T(0), aB0 = T(0), aB1 = T(0);
    if constexpr (NG == 2)
      pdot2_a(aA0, aA1, aB0, aB1, c0.a0, c0.a1, c0.b0, c0.b1, &x[p0], &x[p0 + 16]);
    else
      pdot1_a(aA0, aA1, aB0, aB1, c0.a0, c0.b0, &x[p0]);
    SplitPair<T> nn{};
    if constexpr (pi - PD >= 0)
      nn = split_load_pair<NB, K, 2 * (pi - PD) + 1>(Pj, voff, zero_after(aA0));
    if constexpr (NG == 2)
      pdot2_b(aA0, aA1, aB0, aB1, c0.a0, c0.a1, c0.b0, c0.b1, c0.a2, &x[p0 + 8], &x[p0 + 24],
              &x[p0 + HN]);
    else
      pdot1_b(aA0, aA1, aB0, aB1, c0.a0, c0.b0, c0.a2, &x[p0 + 8], &x[p0 + HN]);
    const T wA = half_pair_sum(aA0 + aA1);
    const T wB = half_pair_sum(aB0 + aB1);
    const T nwA = -(c0.ta * wA);
    const T nwB = -(c0.tb * fma_t(c0.c, nwA, wB));
    if constexpr (NG == 2) {
      pupd2_a(&x[p0], &x[p0 + 16], c0.a0, c0.a1, c0.b0, c0.b1, nwA, nwB);
      pupd2_b(&x[p0 + 8], &x[p0 + 24], &x[p0 + HN], c0.a0, c0.a1, c0.b0, c0.b1, c0.a2, nwA, nwB);
    } else {
      pupd1_a(&x[p0], c0.a0, c0.b0, nwA, nwB);
      pupd1_b(&x[p0 + 8], &x[p0 + HN], c0.a0, c0.b0, c0.a2, nwA, nwB);
    }
    FwdFor<PD - 1>::run([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      buf[i] = buf[i + 1];
    });
    buf[PD - 1] = nn;
  });
}

// Complex counterpart: record values are complex (re, im), reflector o's
// dot product conj(v)^T x and update x += v nw with nw = -tau (dot), each
// complex product as four fp64 FMAs with a broadcast reflector operand.
struct SplitValsC {
  z64 v0, v1, v2, t;
};

template <int NB, int K, int o>
__device__ __forceinline__ SplitValsC split_load_c(const z64* __restrict__ Pj, int voff, int z) {
  using Gm = SplitGeom<NB, K>;
  const z64* __restrict__ rec = Pj + o * Gm::RS + z;
  SplitValsC s;
  s.v0 = rec[voff];
  s.v1 = (Gm::NG == 2) ? rec[voff + 16] : z64{0.0, 0.0};
  s.v2 = (o & 1) ? rec[voff + 16 * Gm::NG] : z64{0.0, 0.0};
  s.t = rec[Gm::HS - 1];
  return s;
}

template <int NB, int K, int PD, int R>
__device__ __forceinline__ void step_split_c(z64 (&x)[R], const z64* __restrict__ Pj, int voff) {
  using Gm = SplitGeom<NB, K>;
  static_assert(R == Gm::R, "window register count");
  static_assert(PD >= 1 && PD <= 4 && PD < K, "prefetch distance 1..4");
  constexpr int HN = Gm::HN, NG = Gm::NG;
  SplitValsC buf[PD];
  FwdFor<PD>::run([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    buf[i] = split_load_c<NB, K, K - 1 - i>(Pj, voff, 0);
  });
  RevFor<K>::run([&](auto oc) {
    constexpr int o = decltype(oc)::value;
    constexpr int p0 = o >> 1;
    const SplitValsC c0 = buf[0];
    double a0r = 0.0, a0i = 0.0, a1r = 0.0, a1i = 0.0;
    if constexpr (NG == 2) {
      cdot_a(a0r, a0i, c0.v0.re, c0.v0.im, &x[p0]);
      cdot_a(a1r, a1i, c0.v1.re, c0.v1.im, &x[p0 + 16]);
    } else {
      cdot_a(a0r, a0i, c0.v0.re, c0.v0.im, &x[p0]);
    }
    SplitValsC nn{};
    if constexpr (o - PD >= 0) nn = split_load_c<NB, K, o - PD>(Pj, voff, zero_after(a0r));
    if constexpr (NG == 2) {
      cdot_b(a0r, a0i, c0.v0.re, c0.v0.im, &x[p0 + 8]);
      cdot_b(a1r, a1i, c0.v1.re, c0.v1.im, &x[p0 + 24]);
    } else {
      cdot_b(a1r, a1i, c0.v0.re, c0.v0.im, &x[p0 + 8]);
    }
    if constexpr ((o & 1) != 0) cdot_x(a0r, a0i, c0.v2.re, c0.v2.im, x[p0 + HN]);
    const double tr = half_pair_sum(a0r + a1r), ti = half_pair_sum(a0i + a1i);
    const double nr = -(c0.t.re * tr - c0.t.im * ti), ni = -(c0.t.re * ti + c0.t.im * tr);
    if constexpr (NG == 2) {
      cupd_a(&x[p0], c0.v0.re, c0.v0.im, nr, ni);
      cupd_a(&x[p0 + 16], c0.v1.re, c0.v1.im, nr, ni);
      cupd_b(&x[p0 + 8], c0.v0.re, c0.v0.im, nr, ni);
      cupd_b(&x[p0 + 24], c0.v1.re, c0.v1.im, nr, ni);
    } else {
      cupd_a(&x[p0], c0.v0.re, c0.v0.im, nr, ni);
      cupd_b(&x[p0 + 8], c0.v0.re, c0.v0.im, nr, ni);
    }
    if constexpr ((o & 1) != 0) cupd_x(x[p0 + HN], c0.v2.re, c0.v2.im, nr, ni);
    FwdFor<PD - 1>::run([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      buf[i] = buf[i + 1];
    });
    buf[PD - 1] = nn;
  });
}

// One tile: chase steps [j0, j1) of block m on stripe c, j1 <= J0(m).
// Row pair (row0+2p, row0+2p+1) of the stripe is the 64 values at
// Qs + (c*rows_pad + row0)*32 + 64p, lane l taking element l.  Block m's
// packed records start at step record Bt[m].
template <typename E, int NB, int K, int PD>
__device__ __forceinline__ void run_split_steps(const E* __restrict__ P,
                                                const int64_t* __restrict__ Bt,
                                                E* __restrict__ Qs, int64_t rows_pad,
                                                int64_t c, int64_t m, int64_t j0, int64_t j1) {
  using Gm = SplitGeom<NB, K>;
  constexpr int R = Gm::R, HN = Gm::HN;
  const int lane = threadIdx.x;
  const int voff = (lane >> 5) * Gm::HS + (lane & 15);
  E* __restrict__ bp = Qs + c * rows_pad * Gm::SW;
  const int64_t s0 = m * K;
  const E* __restrict__ Pm = P + Bt[m] * (K * Gm::RS);
  E x[R];
  for (int64_t j = j0; j < j1; ++j) {
    E* __restrict__ rp = bp + (s0 + 1 + j * NB) * Gm::SW;  // uniform
    if (j == j0) {
#pragma unroll
      for (int p = 0; p < R; ++p) x[p] = rp[p * 64 + lane];
    } else {
#pragma unroll
      for (int p = 0; p < R - HN; ++p) x[p] = x[p + HN];
#pragma unroll
      for (int p = R - HN; p < R; ++p) x[p] = rp[p * 64 + lane];
    }
    if constexpr (std::is_same<E, double>::value || std::is_same<E, float>::value)
      step_split_pair<NB, K, PD>(x, Pm + j * (K * Gm::RS), voff);
    else
      step_split_c<NB, K, PD>(x, Pm + j * (K * Gm::RS), voff);
#pragma unroll
    for (int p = 0; p < HN; ++p) rp[p * 64 + lane] = x[p];
  }
  // window rows NB .. W-1 carried to the next group (or final); the extra row
  // W (upper half of the last register) is not written
  E* __restrict__ rl = bp + (s0 + 1 + (j1 - 1) * NB) * Gm::SW;
#pragma unroll
  for (int p = HN; p < R - 1; ++p) rl[p * 64 + lane] = x[p];
  if (lane < 32) rl[(R - 1) * 64 + lane] = x[R - 1];
}

// Group q (chase steps [qS, min(qS+S, J0))) of block m on stripe c.
template <typename E, int NB, int K, int PD>
__device__ __forceinline__ void run_split_tile(const E* __restrict__ P,
                                               const int64_t* __restrict__ Bt,
                                               E* __restrict__ Qs, int64_t rows_pad, int64_t n,
                                               int64_t c, int64_t m, int64_t q, int64_t S) {
  const int64_t J0 = block_steps(n, NB, K, m);
  const int64_t j0 = q * S;
  const int64_t j1 = (j0 + S < J0) ? j0 + S : J0;
  run_split_steps<E, NB, K, PD>(P, Bt, Qs, rows_pad, c, m, j0, j1);
}

// Stripes c0 .. c0+G-1 of the launch's blocks m0 .. m0+gridDim.x/G-1.
template <typename E, int NB, int K, int OCC, int PD>
__global__ __launch_bounds__(64, OCC) void k_split(const E* __restrict__ P,
                                                   const int64_t* __restrict__ Bt,
                                                   E* __restrict__ Qs, int64_t rows_pad,
                                                   int64_t n, int c0, int G, int M, int t, int m0,
                                                   int S, int xcd) {
  const int b = tile_of((int)blockIdx.x, (int)gridDim.x, xcd);
  const int c = c0 + b % G;
  const int m = m0 + b / G;
  run_split_tile<E, NB, K, PD>(P, Bt, Qs, rows_pad, n, c, m, t - (M - 1 - m), S);
}

// Batched diagonal schedule: launch t runs launch t's tiles of every problem.
template <typename E, int NB, int K, int OCC, int PD>
__global__ __launch_bounds__(64, OCC) void k_split_b(const ProblemDesc* __restrict__ d,
                                                     const DiagEntry* __restrict__ e, int ecount,
                                                     int t, int xcd) {
  const int b = tile_of((int)blockIdx.x, (int)gridDim.x, xcd);
  const DiagEntry& E0 = e[find_by<DiagEntry, &DiagEntry::tile0>(e, ecount, b)];
  const ProblemDesc& D = d[E0.p];
  const int local = b - E0.tile0;
  const int m = E0.m0 + local / D.G;
  run_split_tile<E, NB, K, PD>((const E*)D.P, (const int64_t*)D.Bt, (E*)D.Qs, D.rows_pad, D.n,
                               local % D.G, m, t - (D.M - 1 - m), D.S);
}

// Batched, one launch: workgroup u carries one 32-column stripe of one
// problem through every sweep block, blocks descending and chase steps
// ascending inside a block (the order the diagonal schedule keeps across
// launches: a block's step j needs only the next block's step j done, and
// here that block ran before it in the same wave).  A stripe's window rows
// are read back only by the lanes that wrote them (blocks start K rows apart,
// K even, so a lane keeps its column and row parity), so no workgroup waits
// for another.  Units are numbered problem by problem in the order of the
// descriptor table (the host sorts it by decreasing work), so the dispatcher
// starts the longest units first.  umap (optional) gives the unit of each
// workgroup id, -1 for none: the host deals each problem's stripes to one
// die (workgroup ids go to the dies round robin), so the stripes that read a
// problem's step records run side by side on one die's L2.
template <typename E, int NB, int K, int OCC, int PD>
__global__ __launch_bounds__(64, OCC) void k_split_seq(const ProblemDesc* __restrict__ d,
                                                       int count, const int* __restrict__ umap) {
  const int u = umap ? umap[blockIdx.x] : (int)blockIdx.x;
  if (u < 0) return;
  const ProblemDesc& D = d[find_by<ProblemDesc, &ProblemDesc::unit0>(d, count, u)];
  const int64_t c = u - D.unit0;
  for (int64_t m = D.M - 1; m >= 0; --m)
    run_split_steps<E, NB, K, PD>((const E*)D.P, (const int64_t*)D.Bt, (E*)D.Qs, D.rows_pad, c,
                                  m, 0, block_steps(D.n, NB, K, m));
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// Packed-reflector area of one problem: the step records of every block's
// existing steps back to back (+ 32 values: the extra-segment loads of the
// last record read past it, values never used), then the block offset table
// Bt[0..M).
template <typename E, int NB, int K>
size_t split_rbytes(int64_t n) {
  const int64_t M = (n - 1 + K - 1) / K;
  return align256(((size_t)block_base(n, NB, K, M) * K * SplitGeom<NB, K>::RS + 32) *
                  sizeof(E));
}

template <typename E, int NB, int K>
size_t split_pbytes(int64_t n) {
  const int64_t M = (n - 1 + K - 1) / K;
  return split_rbytes<E, NB, K>(n) + align256((size_t)M * sizeof(int64_t));
}

template <typename E, int NB, int K>
size_t split_workspace(int64_t n, int64_t nev) {
  const DiagPlan pl(n, nev, NB, K, 1, SplitGeom<NB, K>::SW);
  return split_pbytes<E, NB, K>(n) + pl.template qbytes<E>();
}

// Single problem.  ws: a device workspace of at least split_workspace(n, nev)
// bytes that no other work uses while this call's work runs, or null: then
// the workspace is allocated and freed in stream order on st.
template <typename E, int NB, int K, int OCC, int PD>
hipError_t run_split(const void* hh, const void* tau, void* Q, int64_t ldq, int64_t n,
                     int64_t nev, TileOpts opt, hipStream_t st, int num_cu, void* ws_in) {
  using Gm = SplitGeom<NB, K>;
  static const int64_t slots = wave_slots(k_split<E, NB, K, OCC, PD>, num_cu);
  const int64_t S = opt.steps > 0 ? opt.steps : choose_steps(n, nev, NB, K, slots, Gm::SW);
  const DiagPlan pl(n, nev, NB, K, S, Gm::SW);
  const int64_t Jmax = (n - 1 + NB - 1) / NB;
  if (pl.G * pl.M >= INT32_MAX || pl.M * Jmax >= INT32_MAX || n + NB + K >= INT32_MAX)
    return hipErrorInvalidValue;
  const size_t rbytes = split_rbytes<E, NB, K>(n), pbytes = split_pbytes<E, NB, K>(n);
  char* ws = (char*)ws_in;
  if (!ws_in) {
    const hipError_t err = ws_alloc((void**)&ws, pbytes + pl.template qbytes<E>(), st);
    if (err != hipSuccess) return err;
  }
  auto release = [&](hipError_t e) {
    if (!ws_in) {
      const hipError_t e2 = ws_free(ws, st);
      if (e == hipSuccess) e = e2;
    }
    return e;
  };
  E* Pk = (E*)ws;
  int64_t* Bt = (int64_t*)(ws + rbytes);
  E* Qs = (E*)(ws + pbytes);
  const unsigned gt = (unsigned)((nev + 63) / 64);
  hipLaunchKernelGGL((k_pack_split<E, NB, K>), dim3((unsigned)(pl.M * Jmax)), dim3(256), 0, st,
                     (const E*)hh, (const E*)tau, n, Jmax, Pk, Bt);
  hipLaunchKernelGGL((k_to_rows_sw<E, Gm::SW>), dim3((unsigned)(pl.rows_pad / 64), gt), dim3(256), 0,
                     st, (const E*)Q, ldq, n, nev, Qs, pl.rows_pad, pl.G);
  const int ns = (int)std::max<int64_t>(1, std::min<int64_t>(opt.streams, pl.G));
  hipError_t err = hipSuccess;
  ProfScope prof(st, K, S, ns);
  {
    // stripe groups: one launch sequence each, on concurrent streams when
    // more than one (columns are independent; a group's launch tails overlap
    // the other groups' launches)
    StreamFork fork(st, ns);
    if (fork.error() != hipSuccess) return release(fork.error());
    for (int64_t t = 0; t < pl.T; ++t) {
      int64_t m0, cnt;
      pl.active(t, &m0, &cnt);
      if (cnt == 0) continue;
      for (int i = 0; i < ns; ++i) {
        const int64_t c_lo = pl.G * i / ns, gs = pl.G * (i + 1) / ns - c_lo;
        prof.before(fork.stream(i));
        hipLaunchKernelGGL((k_split<E, NB, K, OCC, PD>), dim3((unsigned)(cnt * gs)), dim3(64), 0,
                           fork.stream(i), (const E*)Pk, (const int64_t*)Bt, Qs, pl.rows_pad, n,
                           (int)c_lo, (int)gs, (int)pl.M, (int)t, (int)m0, (int)S, opt.xcd);
        prof.after(fork.stream(i));
      }
    }
    err = fork.join();
  }
  prof.end();
  if (err != hipSuccess) return release(err);
  hipLaunchKernelGGL((k_from_rows_sw<E, Gm::SW>), dim3((unsigned)((n + 63) / 64), gt), dim3(256), 0,
                     st, (const E*)Qs, pl.rows_pad, (E*)Q, ldq, n, nev, pl.G);
  return release(hipGetLastError());
}

template <typename E, int NB, int K, int OCC, int PD>
hipError_t launch_split(const void* hh, const void* tau, void* Q, int64_t ldq, int64_t n,
                        int64_t nev, TileOpts opt, hipStream_t st, int num_cu) {
  return run_split<E, NB, K, OCC, PD>(hh, tau, Q, ldq, n, nev, opt, st, num_cu, nullptr);
}

template <typename E, int NB, int K, int OCC, int PD>
hipError_t launch_split_ws(const void* hh, const void* tau, void* Q, int64_t ldq, int64_t n,
                           int64_t nev, TileOpts opt, hipStream_t st, int num_cu, void* ws) {
  return run_split<E, NB, K, OCC, PD>(hh, tau, Q, ldq, n, nev, opt, st, num_cu, ws);
}

// Modelled times of the two batched schedules, in chase steps of one stripe
// on one wave slot (slots = resident waves of the device).
//  * one launch: each (problem, stripe) unit runs all of its problem's steps
//    plus one step's worth of window load and carry store per sweep block;
//    units start longest first, so the launch takes about max(total / slots,
//    longest unit).
//  * diagonal: launch t of N_t tiles takes ceil(N_t / slots) rounds of S + 1
//    step-units (as in choose_steps), plus half a step per launch for its
//    start.
struct BatchModel {
  double seq = 0.0, diag = 0.0;
};

inline BatchModel batch_model(const std::vector<DiagPlan>& plans, int64_t NB, int64_t K,
                              int64_t slots) {
  BatchModel r;
  double total = 0.0, longest = 0.0;
  int64_t T = 0;
  for (const DiagPlan& pl : plans) {
    const double unit = (double)block_base(pl.n, NB, K, pl.M) + (double)pl.M;
    total += unit * (double)pl.G;
    longest = std::max(longest, unit);
    T = std::max(T, pl.T);
  }
  r.seq = std::max(total / (double)slots, longest);
  for (int64_t t = 0; t < T; ++t) {
    double rounds = 0.0;
    int64_t tiles = 0, smax = 1;
    for (const DiagPlan& pl : plans) {
      int64_t m0, cnt;
      pl.active(t, &m0, &cnt);
      tiles += cnt * pl.G;
      if (cnt) smax = std::max(smax, pl.S);
    }
    if (tiles == 0) continue;
    rounds = (double)((tiles + slots - 1) / slots);
    r.diag += rounds * (double)(smax + 1) + 0.5;
  }
  return r;
}

// Host-side schedule of one batched group: descriptors (device pointers
// bound later), the diagonal schedule's entries, and the workspace layout
// [descriptors | entries | per problem: packed area, stripe copy].
struct SplitBatchPlan {
  std::vector<ProblemDesc> d;
  std::vector<DiagEntry> ent;
  std::vector<int64_t> eoff, etiles;
  std::vector<size_t> pat, qat, rbytes;
  std::vector<int> umap;  // one-launch schedule: unit of each workgroup id (-1: none)
  size_t dbytes = 0, ebytes = 0, ubytes = 0, total = 0, tiles = 0, otiles = 0, ptiles = 0,
         units = 0;
  int64_t T = 0;
  int K = 0;
  bool one_launch = false;
};

// Batched: problems idx[0..cnt) of probs (element type E, semi-bandwidth NB,
// validated by the caller).  Two schedules, the one with the smaller modelled
// time runs (ties and near-ties, within 10 %, go to the single launch):
//  * one launch of k_split_seq, one workgroup per (problem, stripe) unit,
//    problems in order of decreasing work (longest processing time first):
//    for batches of many problems, whose stripes fill the device;
//  * the diagonal schedule of every problem side by side (launch t runs
//    launch t's tiles of every problem): for a few large problems, which need
//    the sweep-block parallelism of the diagonal schedule.
// opt.batch forces one of them; an explicit tile height (opt.steps > 0)
// selects the diagonal schedule.  Returns false if there is nothing to do.
template <typename E, int NB, int K, int OCC, int PD>
hipError_t plan_split_batch(const elpa_hh_problem* probs, const int64_t* idx, int64_t cnt,
                            TileOpts opt, int num_cu, SplitBatchPlan* out) {
  using Gm = SplitGeom<NB, K>;
  static const int64_t slots = wave_slots(k_split_b<E, NB, K, OCC, PD>, num_cu);
  SplitBatchPlan& B = *out;
  B = SplitBatchPlan{};
  B.K = K;
  std::vector<int64_t> live;
  int64_t total_cols = 0;
  for (int64_t i = 0; i < cnt; ++i) {
    const elpa_hh_problem& p = probs[idx[i]];
    if (p.n > 1 && p.nev > 0) {
      live.push_back(idx[i]);
      total_cols += p.nev;
    }
  }
  if (live.empty()) return hipSuccess;
  // work of one stripe unit: step records applied = block_base(M) (equal for
  // every stripe of a problem); stable sort keeps the caller's order on ties
  auto work = [&](int64_t i) {
    const int64_t n = probs[i].n;
    return block_base(n, NB, K, (n - 1 + K - 1) / K);
  };
  std::stable_sort(live.begin(), live.end(),
                   [&](int64_t a, int64_t b) { return work(a) > work(b); });
  std::vector<DiagPlan> plans;
  plans.reserve(live.size());
  for (int64_t i : live) {
    const elpa_hh_problem& p = probs[i];
    const int64_t s = opt.steps > 0 ? opt.steps
                                    : choose_steps(p.n, total_cols, NB, K, slots, Gm::SW);
    plans.emplace_back(p.n, p.nev, NB, K, s, Gm::SW);
  }
  const BatchModel model = batch_model(plans, NB, K, slots);
  B.one_launch = opt.batch == ELPA_BATCH_ONE_LAUNCH ||
                 (opt.batch == ELPA_BATCH_AUTO && opt.steps <= 0 && model.seq <= 1.1 * model.diag);
  B.d.resize(live.size());
  B.pat.resize(live.size());
  B.qat.resize(live.size());
  B.rbytes.resize(live.size());
  size_t off = 0;
  for (size_t i = 0; i < B.d.size(); ++i) {
    const elpa_hh_problem& p = probs[live[i]];
    const DiagPlan& pl = plans[i];
    ProblemDesc& x = B.d[i];
    x.hh = p.hh;
    x.tau = p.tau;
    x.Q = p.Q;
    x.n = p.n;
    x.nev = p.nev;
    x.ldq = p.ldq;
    x.G = (int)pl.G;
    x.GT = (int)((pl.nev + 63) / 64);
    x.M = (int)pl.M;
    x.S = (int)pl.S;
    x.rows_pad = pl.rows_pad;
    x.Jmax = (pl.n - 1 + NB - 1) / NB;
    x.tile0 = (int)B.tiles;
    x.otile0 = (int)B.otiles;
    x.ptile0 = (int)B.ptiles;
    x.unit0 = (int)B.units;
    B.tiles += (size_t)(pl.rows_pad / 64 * x.GT);
    B.otiles += (size_t)((pl.n + 63) / 64 * x.GT);
    B.ptiles += (size_t)(pl.M * x.Jmax);
    B.units += (size_t)pl.G;
    B.pat[i] = off;
    B.rbytes[i] = split_rbytes<E, NB, K>(pl.n);
    off += split_pbytes<E, NB, K>(pl.n);
    B.qat[i] = off;
    off += pl.template qbytes<E>();
    B.T = std::max(B.T, pl.T);
  }
  B.eoff.assign((size_t)B.T + 1, 0);
  B.etiles.assign((size_t)B.T, 0);
  if (!B.one_launch) {
    for (int64_t t = 0; t < B.T; ++t) {
      B.eoff[(size_t)t] = (int64_t)B.ent.size();
      int64_t tl = 0;
      for (size_t i = 0; i < B.d.size(); ++i) {
        int64_t m0, c;
        plans[i].active(t, &m0, &c);
        if (c == 0) continue;
        B.ent.push_back(DiagEntry{(int)i, (int)m0, (int)c, (int)tl});
        tl += c * plans[i].G;
      }
      B.etiles[(size_t)t] = tl;
    }
    B.eoff[(size_t)B.T] = (int64_t)B.ent.size();
  }
  if (B.tiles >= (size_t)INT32_MAX || B.otiles >= (size_t)INT32_MAX ||
      B.ptiles >= (size_t)INT32_MAX || B.units >= (size_t)INT32_MAX)
    return hipErrorInvalidValue;
  for (int64_t x : B.etiles)
    if (x >= INT32_MAX) return hipErrorInvalidValue;
  if (B.one_launch && opt.order != ELPA_ORDER_LINEAR) {
    // deal whole problems to the dies, longest first, each to the die with
    // the least work so far; die x runs workgroup ids x, x + dies, ...
    constexpr int dies = 8;
    std::vector<std::vector<int>> lists(dies);
    std::vector<double> load(dies, 0.0);
    for (size_t i = 0; i < B.d.size(); ++i) {
      const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      load[(size_t)x] += (double)B.d[i].G * (double)work(live[i]);
      for (int c = 0; c < B.d[i].G; ++c) lists[(size_t)x].push_back(B.d[i].unit0 + c);
    }
    size_t len = 0;
    for (const auto& l : lists) len = std::max(len, l.size());
    if (len * dies >= (size_t)INT32_MAX) return hipErrorInvalidValue;
    B.umap.assign(len * dies, -1);
    for (int x = 0; x < dies; ++x)
      for (size_t i = 0; i < lists[(size_t)x].size(); ++i)
        B.umap[i * dies + (size_t)x] = lists[(size_t)x][i];
  }
  B.dbytes = align256(B.d.size() * sizeof(ProblemDesc));
  B.ebytes = align256(std::max<size_t>(1, B.ent.size()) * sizeof(DiagEntry));
  B.ubytes = align256(B.umap.size() * sizeof(int));
  B.total = B.dbytes + B.ebytes + B.ubytes + off;
  return hipSuccess;
}

// Device addresses of the plan's areas in a workspace of B.total bytes.
inline void bind_split_batch(SplitBatchPlan& B, char* ws) {
  for (size_t i = 0; i < B.d.size(); ++i) {
    char* area = ws + B.dbytes + B.ebytes + B.ubytes;
    B.d[i].P = area + B.pat[i];
    B.d[i].Bt = area + B.pat[i] + B.rbytes[i];
    B.d[i].Qs = area + B.qat[i];
  }
}

// The launches of a bound plan whose descriptor and entry tables are in the
// workspace: packing, layout conversion, the schedule, conversion back.
template <typename E, int NB, int K, int OCC, int PD>
void launch_split_batch(const SplitBatchPlan& B, const char* ws, int xcd, hipStream_t st) {
  using Gm = SplitGeom<NB, K>;
  const ProblemDesc* dd = (const ProblemDesc*)ws;
  const DiagEntry* de = (const DiagEntry*)(ws + B.dbytes);
  const int count = (int)B.d.size();
  hipLaunchKernelGGL((k_pack_split_b<E, NB, K>), dim3((unsigned)B.ptiles), dim3(256), 0, st, dd,
                     count);
  hipLaunchKernelGGL((k_to_rows_sw_b<E, Gm::SW>), dim3((unsigned)B.tiles), dim3(256), 0, st, dd,
                     count);
  {
    ProfScope prof(st, K, 0);
    if (B.one_launch) {
      prof.before(st);
      const int* um = B.umap.empty() ? nullptr : (const int*)(ws + B.dbytes + B.ebytes);
      const size_t grid = B.umap.empty() ? B.units : B.umap.size();
      hipLaunchKernelGGL((k_split_seq<E, NB, K, OCC, PD>), dim3((unsigned)grid), dim3(64), 0, st,
                         dd, count, um);
      prof.after(st);
    } else {
      for (int64_t t = 0; t < B.T; ++t) {
        const int64_t ne = B.eoff[(size_t)t + 1] - B.eoff[(size_t)t];
        if (ne == 0) continue;
        prof.before(st);
        hipLaunchKernelGGL((k_split_b<E, NB, K, OCC, PD>), dim3((unsigned)B.etiles[(size_t)t]),
                           dim3(64), 0, st, dd, de + B.eoff[(size_t)t], (int)ne, (int)t, xcd);
        prof.after(st);
      }
    }
  }
  hipLaunchKernelGGL((k_from_rows_sw_b<E, Gm::SW>), dim3((unsigned)B.otiles), dim3(256), 0, st,
                     dd, count);
}

// Batched call: plan, stream-ordered workspace, tables staged through pinned
// host memory, launches, workspace freed in stream order.
template <typename E, int NB, int K, int OCC, int PD>
hipError_t launch_split_batched(const elpa_hh_problem* probs, const int64_t* idx, int64_t cnt,
                                TileOpts opt, hipStream_t st, int num_cu) {
  SplitBatchPlan B;
  hipError_t err = plan_split_batch<E, NB, K, OCC, PD>(probs, idx, cnt, opt, num_cu, &B);
  if (err != hipSuccess || B.d.empty()) return err;
  char* ws = nullptr;
  err = ws_alloc((void**)&ws, B.total, st);
  if (err != hipSuccess) return err;
  bind_split_batch(B, ws);
  int dev = 0;
  (void)hipGetDevice(&dev);
  PinnedStaging& stage = PinnedStaging::for_device(dev);
  err = stage.upload(ws, B.d.data(), B.d.size() * sizeof(ProblemDesc), st);
  if (err == hipSuccess && !B.ent.empty())
    err = stage.upload(ws + B.dbytes, B.ent.data(), B.ent.size() * sizeof(DiagEntry), st);
  if (err == hipSuccess && !B.umap.empty())
    err = stage.upload(ws + B.dbytes + B.ebytes, B.umap.data(), B.umap.size() * sizeof(int), st);
  if (err != hipSuccess) {
    (void)ws_free(ws, st);
    return err;
  }
  launch_split_batch<E, NB, K, OCC, PD>(B, ws, opt.xcd, st);
  err = hipGetLastError();
  const hipError_t e2 = ws_free(ws, st);
  return err != hipSuccess ? err : e2;
}

// Prepared group (elpa_hh_batch_create): the workspace and tables live on the
// device for the handle's lifetime; run() only launches.  A single problem
// runs the single-call path (stripe groups on library streams) on the owned
// workspace; several run the batched schedule.
template <typename E, int NB, int K, int OCC, int PD>
class SplitPrepared : public PreparedGroup {
 public:
  ~SplitPrepared() override {
    if (ws_) (void)hipFree(ws_);
  }
  hipError_t init(const elpa_hh_problem* probs, const int64_t* idx, int64_t cnt, TileOpts opt,
                  int num_cu) {
    opt_ = opt;
    num_cu_ = num_cu;
    int live = 0;
    for (int64_t i = 0; i < cnt; ++i)
      if (probs[idx[i]].n > 1 && probs[idx[i]].nev > 0) {
        ++live;
        single_ = probs[idx[i]];
      }
    if (live == 0) return hipSuccess;
    if (live == 1) {
      one_ = true;
      bytes_ = split_workspace<E, NB, K>(single_.n, single_.nev);
      return alloc(bytes_);
    }
    hipError_t err = plan_split_batch<E, NB, K, OCC, PD>(probs, idx, cnt, opt, num_cu, &B_);
    if (err != hipSuccess) return err;
    bytes_ = B_.total;
    err = alloc(bytes_);
    if (err != hipSuccess) return err;
    bind_split_batch(B_, (char*)ws_);
    err = hipMemcpy(ws_, B_.d.data(), B_.d.size() * sizeof(ProblemDesc), hipMemcpyHostToDevice);
    if (err == hipSuccess && !B_.ent.empty())
      err = hipMemcpy((char*)ws_ + B_.dbytes, B_.ent.data(), B_.ent.size() * sizeof(DiagEntry),
                      hipMemcpyHostToDevice);
    if (err == hipSuccess && !B_.umap.empty())
      err = hipMemcpy((char*)ws_ + B_.dbytes + B_.ebytes, B_.umap.data(),
                      B_.umap.size() * sizeof(int), hipMemcpyHostToDevice);
    return err;
  }
  hipError_t run(hipStream_t st) override {
    if (!ws_) return hipSuccess;
    if (one_)
      return run_split<E, NB, K, OCC, PD>(single_.hh, single_.tau, single_.Q, single_.ldq,
                                          single_.n, single_.nev, opt_, st, num_cu_, ws_);
    launch_split_batch<E, NB, K, OCC, PD>(B_, (const char*)ws_, opt_.xcd, st);
    return hipGetLastError();
  }
  size_t bytes() const override { return bytes_; }

 private:
  hipError_t alloc(size_t b) {
    size_t tot = 0;
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceTotalMem(&tot, dev) == hipSuccess &&
        tot && b > tot)
      return hipErrorOutOfMemory;
    const hipError_t e = hipMalloc(&ws_, b);
    if (e != hipSuccess) {
      ws_ = nullptr;
      (void)hipGetLastError();
    }
    return e;
  }
  SplitBatchPlan B_;
  elpa_hh_problem single_{};
  bool one_ = false;
  TileOpts opt_{};
  int num_cu_ = 0;
  void* ws_ = nullptr;
  size_t bytes_ = 0;
};

template <typename E, int NB, int K, int OCC, int PD>
hipError_t prepare_split(const elpa_hh_problem* probs, const int64_t* idx, int64_t cnt,
                         TileOpts opt, int num_cu, PreparedGroup** out) {
  auto* g = new SplitPrepared<E, NB, K, OCC, PD>();
  const hipError_t err = g->init(probs, idx, cnt, opt, num_cu);
  if (err != hipSuccess) {
    delete g;
    *out = nullptr;
    return err;
  }
  *out = g;
  return hipSuccess;
}

}  // namespace ehh
