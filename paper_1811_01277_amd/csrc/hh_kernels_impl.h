// HIP kernels (gfx950) of the tridiagonal->band eigenvector back-transformation
//
//     Q <- H(0,0) H(0,1) ... H(n-2, J-1) Q,      H(s,j) = I - tau v v^H,
//
// the two-stage solver's first back-transformation (Kus et al., Sec. 2; the
// compute-heavy part of the back-transformation singled out in Sec. 3.1).
//
// Stripe path
// -----------
// 1. Q (column major) is copied into a stripe-major workspace Qs: each
//    64-column stripe (G = ceil(nev/64) of them) is a contiguous row-major
//    block with zero rows past n, enough for the deepest window.  A wave64
//    lane owns one column, so a row of a stripe is one 512-byte coalesced
//    access, the row stride is a compile-time constant, and no load or store
//    needs a bounds check.
// 2. Sweeps are grouped into blocks of K consecutive sweeps [mK, mK+K-1]
//    (m = 0..M-1).  Block m slides a window of W = NB+K-1 rows of a stripe
//    down the matrix, one chase step j at a time; at each step it applies the
//    K reflectors (s, j) of the block, largest s first, to the window held in
//    VGPRs, writes the NB rows that are final for the block and reads NB new
//    ones (2*NB*K FMAs per lane per 2*NB row transfers).
// 3. Order.  Two reflectors (a, j), (c, j') with a > c share rows only if
//    a - c >= NB*(j'-j-1)+1, so blocks may run from the top (largest sweeps)
//    down with chase steps ascending inside a block, and block m at step j
//    only needs block m+1 to have finished its step j.  The result equals
//    strict reverse generation order up to the rounding of the dot products.
// 4. Schedule (no synchronisation inside a launch).  A tile is (stripe c,
//    block m, group q of S consecutive chase steps).  Launch t runs every
//    tile with (M-1-m) + q = t.  Block m's group q then runs after block
//    m+1's group q (launch t-1), which covers every row it needs, and the
//    tiles of one launch touch disjoint rows of a stripe: block m's group q
//    ends at row s0+K-1+(q+1)*S*NB, block m+1's group q+1 starts at row
//    s0+K+1+(q+1)*S*NB, block m-1's group q-1 ends at row s0-1+q*S*NB and
//    block m's group q starts at s0+1+q*S*NB.  Kernel boundaries give all
//    ordering and visibility; a tile that ends mid-block writes its K-1
//    carried rows back and the next group reloads them.  Launch count is
//    about M + ceil(J0/S); S trades launches and window reloads for
//    parallelism (tiles per launch ~ G * min(M, J0/S)).
// 5. Qs is copied back into Q.
// 6. Batched form: launch t runs the tiles of launch t of every problem of
//    the batch (one element type and NB per launch sequence).
//
// Reference path: any nbw, one reflector at a time, column-major in place.
#pragma once

#include "hh_common.h"
#include "hh_dispatch.h"
#include "hh_dpp.h"
#include "hh_sched.h"

namespace ehh {

// ---------------------------------------------------------------------------
// Reference kernel: strict reverse generation order, one lane per column,
// the column kept in global memory.
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



template <typename E>
__device__ __forceinline__ void to_rows_tile(const E* __restrict__ Q, int64_t ldq, int64_t n,
                                             int64_t nev, E* __restrict__ Qs, int64_t rows_pad,
                                             int64_t rt, int64_t c, E (*tile)[65]) {
  const int64_t r0 = rt * 64, c0 = c * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int cc = ty; cc < 64; cc += 4) {
    const int64_t r = r0 + tx, col = c0 + cc;
    tile[cc][tx] = (r < n && col < nev) ? Q[r + col * ldq] : Ops<E>::zero();
  }
  __syncthreads();
  E* __restrict__ dst = Qs + c * rows_pad * 64;
  for (int rr = ty; rr < 64; rr += 4) {
    const int64_t r = r0 + rr;
    if (r < rows_pad) dst[r * 64 + tx] = tile[tx][rr];
  }
}

template <typename E>
__device__ __forceinline__ void from_rows_tile(const E* __restrict__ Qs, int64_t rows_pad,
                                               E* __restrict__ Q, int64_t ldq, int64_t n,
                                               int64_t nev, int64_t rt, int64_t c,
                                               E (*tile)[65]) {
  const int64_t r0 = rt * 64, c0 = c * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const E* __restrict__ src = Qs + c * rows_pad * 64;
  for (int rr = ty; rr < 64; rr += 4) {
    const int64_t r = r0 + rr;
    if (r < n) tile[rr][tx] = src[r * 64 + tx];
  }
  __syncthreads();
  for (int cc = ty; cc < 64; cc += 4) {
    const int64_t r = r0 + tx, col = c0 + cc;
    if (r < n && col < nev) Q[r + col * ldq] = tile[tx][cc];
  }
}

template <typename E>
__global__ __launch_bounds__(256) void k_to_rows_b(const ProblemDesc* __restrict__ d, int count) {
  __shared__ E tile[64][65];
  const int t = (int)blockIdx.x;
  const int p = find_by<ProblemDesc, &ProblemDesc::tile0>(d, count, t);
  const ProblemDesc& P = d[p];
  const int local = t - P.tile0;
  to_rows_tile<E>((const E*)P.Q, P.ldq, P.n, P.nev, (E*)P.Qs, P.rows_pad, local / P.GT,
                  local % P.GT, tile);
}

template <typename E>
__global__ __launch_bounds__(256) void k_from_rows_b(const ProblemDesc* __restrict__ d,
                                                     int count) {
  __shared__ E tile[64][65];
  const int t = (int)blockIdx.x;
  const int p = find_by<ProblemDesc, &ProblemDesc::otile0>(d, count, t);
  const ProblemDesc& P = d[p];
  const int local = t - P.otile0;
  from_rows_tile<E>((const E*)P.Qs, P.rows_pad, (E*)P.Q, P.ldq, P.n, P.nev, local / P.GT,
                    local % P.GT, tile);
}

// ---------------------------------------------------------------------------
// Layout conversion between Q (column major, ldq) and the stripe-major
// workspace Qs: stripe c (columns 64c..64c+63) is a contiguous rows_pad x 64
// row-major block, element (r, 64c+l) at Qs[(c*rows_pad + r)*64 + l].
// 64x64 tiles through LDS; padding rows and columns are written as zeros.
// ---------------------------------------------------------------------------
template <typename E>
__global__ __launch_bounds__(256) void k_to_rows(const E* __restrict__ Q, int64_t ldq, int64_t n,
                                                 int64_t nev, E* __restrict__ Qs,
                                                 int64_t rows_pad) {
  __shared__ E tile[64][65];
  to_rows_tile<E>(Q, ldq, n, nev, Qs, rows_pad, blockIdx.x, blockIdx.y, tile);
}

template <typename E>
__global__ __launch_bounds__(256) void k_from_rows(const E* __restrict__ Qs, int64_t rows_pad,
                                                   E* __restrict__ Q, int64_t ldq, int64_t n,
                                                   int64_t nev) {
  __shared__ E tile[64][65];
  from_rows_tile<E>(Qs, rows_pad, Q, ldq, n, nev, blockIdx.x, blockIdx.y, tile);
}

// ---------------------------------------------------------------------------
// Reflector streaming helpers.
// ---------------------------------------------------------------------------
// Reflector values travel through SGPRs in chunks of CH elements, with a
// software pipeline of one chunk: the scalar loads of chunk q+1 are issued
// right after the first FMA of chunk q and consumed by chunk q+1.  LLVM may
// move loads of read-only memory anywhere; after() gives the next address a
// (zero) data dependence on an FMA result of the current chunk, so the loads
// stay where they are issued instead of being hoisted en masse (which would
// overflow the 102 SGPRs and spill).
template <typename E>
struct ChunkSize {
  static constexpr int value = (sizeof(E) >= 16) ? 4 : (sizeof(E) == 8 ? 8 : 16);
};

template <typename E, int CH>
struct Chunk {
  E v[CH];
};

template <typename E, int CH>
__device__ __forceinline__ Chunk<E, CH> load_chunk(const E* __restrict__ p) {
  Chunk<E, CH> c;
#pragma unroll
  for (int k = 0; k < CH; ++k) c.v[k] = p[k];
  return c;
}


template <typename E, typename D>
__device__ __forceinline__ const E* after(const E* p, D dep) {
  return p + zero_after(dep);
}

// Apply H = I - t v v^H to window rows [o, o+NB) of every lane's column.
// On entry cur holds the first CH elements of v (from vd); on exit it holds
// the first CH elements at vnext (the next reflector).  vd and vu point to
// the same values (vu through a separate read-only kernel argument, so the
// two passes' loads are not merged and v is not held in SGPRs between them).
template <typename E, int NB, int W>
__device__ __forceinline__ void apply_reflector(E (&x)[W], int o, const E* __restrict__ vd,
                                                const E* __restrict__ vu,
                                                const E* __restrict__ vnext, E t,
                                                Chunk<E, ChunkSize<E>::value>& cur) {
  using O = Ops<E>;
  constexpr int CH = ChunkSize<E>::value;
  constexpr int NC = NB / CH;
  static_assert(NB % CH == 0, "NB must be a multiple of the chunk size");
  E a0 = O::zero(), a1 = O::zero(), a2 = O::zero(), a3 = O::zero();
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const int b = o + q * CH;
    O::dot(a0, cur.v[0], x[b]);
    const E* np = (q + 1 < NC) ? vd + (q + 1) * CH : vu;
    const Chunk<E, CH> nxt = load_chunk<E, CH>(after(np, a0));
#pragma unroll
    for (int k = 1; k < CH; ++k) {
      E& acc = (k & 3) == 0 ? a0 : ((k & 3) == 1 ? a1 : ((k & 3) == 2 ? a2 : a3));
      O::dot(acc, cur.v[k], x[b + k]);
    }
    cur = nxt;
  }
  const E w = O::scale(O::add(O::add(a0, a1), O::add(a2, a3)), t);
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const int b = o + q * CH;
    O::axpy(x[b], cur.v[0], w);
    const E* np = (q + 1 < NC) ? vu + (q + 1) * CH : vnext;
    const Chunk<E, CH> nxt = load_chunk<E, CH>(after(np, x[b]));
#pragma unroll
    for (int k = 1; k < CH; ++k) O::axpy(x[b + k], cur.v[k], w);
    cur = nxt;
  }
  // keep successive reflectors from being interleaved by the scheduler
  __builtin_amdgcn_sched_barrier(0);
}


// ---------------------------------------------------------------------------
// One chase step of one block: apply the K reflectors (s0+o, j), o = K-1..0,
// to the window x (rows row0 .. row0+W-1 of the lane's column).  A reflector
// that does not exist is applied as slot 0 with tau = 0 (exact no-op on finite
// data), which keeps the unrolled step free of branches.
// ---------------------------------------------------------------------------
template <typename E, int NB, int K>
struct StepSmem {
  static constexpr int W = NB + K - 1;
  static __device__ __forceinline__ void run(E (&x)[W], const E* __restrict__ hh,
                                             const E* __restrict__ hh2,
                                             const E* __restrict__ tau, int64_t s0, int64_t s1,
                                             int64_t j, int64_t n, int64_t ctot) {
    using O = Ops<E>;
    auto slot_of = [&](int o) -> int64_t {
      const int64_t s = s0 + o;
      const bool ok = (s <= s1) && (s + 1 + j * NB < n);
      return ok ? ctot - csum(n - 1 - s, NB) + j : -1;
    };
    int64_t sl = slot_of(K - 1);
    Chunk<E, ChunkSize<E>::value> cur =
        load_chunk<E, ChunkSize<E>::value>(hh + (sl < 0 ? 0 : sl) * NB);
    RevFor<K>::run([&](auto oc) {
      constexpr int o = decltype(oc)::value;
      const int64_t sn = (o > 0) ? slot_of(o - 1) : -1;
      const int64_t su = sl < 0 ? 0 : sl;
      const E t = sl < 0 ? O::zero() : tau[su];
      apply_reflector<E, NB, W>(x, o, hh + su * NB, hh2 + su * NB, hh + (sn < 0 ? 0 : sn) * NB,
                                t, cur);
      sl = sn;
    });
  }
};

// fp64: the reflector v (NB values) lives in NG = NB/16 VGPR pairs, lane l
// holding v[16g + l%16] in pair g, and is fed to the FMAs by DPP
// row_newbcast; v and tau are vector-loaded one reflector ahead.  NG
// independent accumulators, one per 16-value segment.
template <int NB, int K>
struct StepDpp {
  static constexpr int W = NB + K - 1;
  static constexpr int NG = NB / 16;
  static_assert(NB == 32 || NB == 64, "DPP step supports NB = 32, 64");
  static __device__ __forceinline__ void run(double (&x)[W], const double* __restrict__ hh,
                                             const double* __restrict__,
                                             const double* __restrict__ tau, int64_t s0,
                                             int64_t s1, int64_t j, int64_t n, int64_t ctot) {
    const int l16 = threadIdx.x & 15;
    auto slot_of = [&](int o) -> int64_t {
      const int64_t s = s0 + o;
      const bool ok = (s <= s1) && (s + 1 + j * NB < n);
      return ok ? ctot - csum(n - 1 - s, NB) + j : -1;
    };
    double V[NG], T;
    {
      const int64_t sl = slot_of(K - 1);
      const int64_t su = sl < 0 ? 0 : sl;
      const double* __restrict__ p = hh + su * NB + l16;
#pragma unroll
      for (int g = 0; g < NG; ++g) V[g] = p[16 * g];
      const double tl = tau[su];
      T = sl < 0 ? 0.0 : tl;
    }
    RevFor<K>::run([&](auto oc) {
      constexpr int o = decltype(oc)::value;
      const int64_t sn = (o > 0) ? slot_of(o - 1) : -1;
      const int64_t snu = sn < 0 ? 0 : sn;
      double Vn[NG], Tn = 0.0;
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      FwdFor<16>::run([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        if constexpr (NG == 4) {
          dpp_dot4<i>(a0, a1, a2, a3, V[0], V[1], V[2], V[3], &x[o + i], &x[o + 16 + i],
                      &x[o + 32 + i], &x[o + 48 + i]);
        } else {
          dpp_dot2<i>(a0, a1, V[0], V[1], &x[o + i], &x[o + 16 + i]);
        }
        if constexpr (i == 0) {
          // prefetch the next reflector; its address depends on a0 so the
          // loads are issued here and not hoisted
          const int z = zero_after(a0);
          const double* __restrict__ p = hh + snu * NB + z + l16;
#pragma unroll
          for (int g = 0; g < NG; ++g) Vn[g] = p[16 * g];
          const double tl = tau[snu + z];
          Tn = sn < 0 ? 0.0 : tl;
        }
      });
      const double nw = -(T * ((a0 + a1) + (a2 + a3)));
      FwdFor<16>::run([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        if constexpr (NG == 4) {
          dpp_upd4<i>(x[o + i], x[o + 16 + i], x[o + 32 + i], x[o + 48 + i], V[0], V[1], V[2],
                      V[3], nw);
        } else {
          dpp_upd2<i>(x[o + i], x[o + 16 + i], V[0], V[1], nw);
        }
      });
#pragma unroll
      for (int g = 0; g < NG; ++g) V[g] = Vn[g];
      T = Tn;
    });
  }
};

template <typename E, int NB, int K>
struct StepFor {
  using type = StepSmem<E, NB, K>;
};
template <int NB, int K>
struct StepFor<double, NB, K> {
  using type = StepDpp<NB, K>;
};

// ---------------------------------------------------------------------------
// One tile: group q (chase steps [qS, min(qS+S, J0))) of block m on stripe c.
//   Qs   stripe-major workspace, row r of stripe c at Qs + (c*rows_pad + r)*64
// ---------------------------------------------------------------------------
template <typename E, int NB, int K>
__device__ __forceinline__ void run_tile(const E* __restrict__ hh, const E* __restrict__ hh2,
                                         const E* __restrict__ tau, E* __restrict__ Qs,
                                         int64_t rows_pad, int64_t n, int64_t c, int64_t m,
                                         int64_t q, int64_t S) {
  constexpr int W = NB + K - 1;
  const int lane = threadIdx.x;
  const int64_t ctot = csum(n - 1, NB);
  E x[W];
  // uniform base of the stripe; row r of the lane's column is bp[r*64 + lane]
  E* __restrict__ bp = Qs + c * rows_pad * 64;
  const int64_t s0 = m * K;
  const int64_t s1 = (s0 + K - 1 < n - 2) ? s0 + K - 1 : n - 2;
  const int64_t J0 = (n - 1 - s0 + NB - 1) / NB;
  const int64_t j0 = q * S;
  const int64_t j1 = (j0 + S < J0) ? j0 + S : J0;
  for (int64_t j = j0; j < j1; ++j) {
    const int64_t row0 = s0 + 1 + j * NB;
    E* __restrict__ rp = bp + row0 * 64;  // uniform
    if (j == j0) {
#pragma unroll
      for (int i = 0; i < W; ++i) x[i] = rp[i * 64 + lane];
    } else {
#pragma unroll
      for (int i = 0; i < K - 1; ++i) x[i] = x[i + NB];
#pragma unroll
      for (int i = K - 1; i < W; ++i) x[i] = rp[i * 64 + lane];
    }
    StepFor<E, NB, K>::type::run(x, hh, hh2, tau, s0, s1, j, n, ctot);
#pragma unroll
    for (int i = 0; i < NB; ++i) rp[i * 64 + lane] = x[i];
  }
  // rows carried to the next group (or final after the block's last step)
  E* __restrict__ rl = bp + (s0 + 1 + (j1 - 1) * NB) * 64;
#pragma unroll
  for (int i = NB; i < W; ++i) rl[i * 64 + lane] = x[i];
}

// ---------------------------------------------------------------------------
// Diagonal-schedule kernels.  One problem: blockIdx.x = (block m0+i, stripe
// c) over the launch's blocks; group q = t - (M-1-m).  Batched: the launch's
// entries map blockIdx.x to (problem, block, stripe).  hh2 == hh (see
// apply_reflector).
// ---------------------------------------------------------------------------
template <typename E, int NB, int K, int OCC>
__global__ __launch_bounds__(64, OCC) void k_diag(const E* __restrict__ hh,
                                                  const E* __restrict__ hh2,
                                                  const E* __restrict__ tau, E* __restrict__ Qs,
                                                  int64_t rows_pad, int64_t n, int c0, int G,
                                                  int M, int t, int m0, int S, int xcd) {
  const int b = tile_of((int)blockIdx.x, (int)gridDim.x, xcd);
  const int c = c0 + b % G;
  const int m = m0 + b / G;
  const int q = t - (M - 1 - m);
  run_tile<E, NB, K>(hh, hh2, tau, Qs, rows_pad, n, c, m, q, S);
}

template <typename E, int NB, int K, int OCC>
__global__ __launch_bounds__(64, OCC) void k_diag_b(const ProblemDesc* __restrict__ d,
                                                    const DiagEntry* __restrict__ e, int ecount,
                                                    int t, int xcd) {
  const int b = tile_of((int)blockIdx.x, (int)gridDim.x, xcd);
  const int ei = find_by<DiagEntry, &DiagEntry::tile0>(e, ecount, b);
  const DiagEntry& E0 = e[ei];
  const ProblemDesc& P = d[E0.p];
  const int local = b - E0.tile0;
  const int c = local % P.G;
  const int m = E0.m0 + local / P.G;
  const int q = t - (P.M - 1 - m);
  run_tile<E, NB, K>((const E*)P.hh, (const E*)P.hh, (const E*)P.tau, (E*)P.Qs, P.rows_pad, P.n,
                     c, m, q, P.S);
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


template <typename E, int NB, int K, int OCC>
hipError_t launch_diag(const void* hh, const void* tau, void* Q, int64_t ldq, int64_t n,
                       int64_t nev, TileOpts opt, hipStream_t st, int num_cu) {
  static const int64_t slots = wave_slots(k_diag<E, NB, K, OCC>, num_cu);
  const int64_t S = opt.steps > 0 ? opt.steps : choose_steps(n, nev, NB, K, slots, 64);
  const DiagPlan pl(n, nev, NB, K, S);
  if (pl.G * pl.M >= INT32_MAX || n + NB + K >= INT32_MAX) return hipErrorInvalidValue;
  E* Qs = nullptr;
  hipError_t err = ws_alloc((void**)&Qs, pl.template qbytes<E>(), st);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_to_rows<E>, dim3((unsigned)(pl.rows_pad / 64), (unsigned)pl.G), dim3(256),
                     0, st, (const E*)Q, ldq, n, nev, Qs, pl.rows_pad);
  const int ns = (int)std::max<int64_t>(1, std::min<int64_t>(opt.streams, pl.G));
  ProfScope prof(st, K, S, ns);
  {
    // stripe groups on concurrent streams (see the split kernel's launcher)
    StreamFork fork(st, ns);
    if (fork.error() != hipSuccess) {
      (void)ws_free(Qs, st);
      return fork.error();
    }
    for (int64_t t = 0; t < pl.T; ++t) {
      int64_t m0, cnt;
      pl.active(t, &m0, &cnt);
      if (cnt == 0) continue;
      for (int i = 0; i < ns; ++i) {
        const int64_t c_lo = pl.G * i / ns, gs = pl.G * (i + 1) / ns - c_lo;
        prof.before(fork.stream(i));
        hipLaunchKernelGGL((k_diag<E, NB, K, OCC>), dim3((unsigned)(cnt * gs)), dim3(64), 0,
                           fork.stream(i), (const E*)hh, (const E*)hh, (const E*)tau, Qs,
                           pl.rows_pad, n, (int)c_lo, (int)gs, (int)pl.M, (int)t, (int)m0, (int)S,
                           opt.xcd);
        prof.after(fork.stream(i));
      }
    }
    err = fork.join();
  }
  prof.end();
  if (err != hipSuccess) {
    (void)ws_free(Qs, st);
    return err;
  }
  hipLaunchKernelGGL(k_from_rows<E>, dim3((unsigned)((n + 63) / 64), (unsigned)pl.G), dim3(256),
                     0, st, (const E*)Qs, pl.rows_pad, (E*)Q, ldq, n, nev);
  err = hipGetLastError();
  const hipError_t e2 = ws_free(Qs, st);
  return err != hipSuccess ? err : e2;
}

// Batched launch: problems idx[0..cnt) of probs (all of element type E and
// semi-bandwidth NB, validated by the caller): the diagonal schedules of all
// problems run side by side, launch t holding launch t of every problem.
template <typename E, int NB, int K, int OCC>
hipError_t launch_diag_batched(const elpa_hh_problem* probs, const int64_t* idx, int64_t cnt,
                               TileOpts opt, hipStream_t st, int num_cu) {
  const int64_t S = opt.steps;
  static const int64_t slots = wave_slots(k_diag_b<E, NB, K, OCC>, num_cu);
  std::vector<ProblemDesc> d;
  std::vector<DiagPlan> plans;
  d.reserve((size_t)cnt);
  plans.reserve((size_t)cnt);
  int64_t total_cols = 0;
  for (int64_t i = 0; i < cnt; ++i) {
    const elpa_hh_problem& p = probs[idx[i]];
    if (p.n <= 1 || p.nev == 0) continue;
    total_cols += p.nev;
  }
  for (int64_t i = 0; i < cnt; ++i) {
    const elpa_hh_problem& p = probs[idx[i]];
    if (p.n <= 1 || p.nev == 0) continue;
    // all problems share the launch slots: size S from the batch's columns
    const int64_t s = S > 0 ? S : choose_steps(p.n, total_cols, NB, K, slots, 64);
    plans.emplace_back(p.n, p.nev, NB, K, s);
    ProblemDesc x{};
    x.hh = p.hh;
    x.tau = p.tau;
    x.Q = p.Q;
    x.n = p.n;
    x.nev = p.nev;
    x.ldq = p.ldq;
    d.push_back(x);
  }
  if (d.empty()) return hipSuccess;
  size_t qoff = 0, tiles = 0, otiles = 0;
  int64_t T = 0;
  std::vector<size_t> qat(d.size());
  for (size_t i = 0; i < d.size(); ++i) {
    const DiagPlan& pl = plans[i];
    d[i].G = (int)pl.G;
    d[i].GT = (int)pl.G;  // 64-column stripes: one conversion tile column per stripe
    d[i].M = (int)pl.M;
    d[i].S = (int)pl.S;
    d[i].rows_pad = pl.rows_pad;
    d[i].tile0 = (int)tiles;
    d[i].otile0 = (int)otiles;
    tiles += (size_t)(pl.rows_pad / 64 * pl.G);
    otiles += (size_t)((pl.n + 63) / 64 * pl.G);
    qat[i] = qoff;
    qoff += pl.template qbytes<E>();
    T = std::max(T, pl.T);
  }
  // schedule entries of every launch, concatenated
  std::vector<DiagEntry> ent;
  std::vector<int64_t> eoff((size_t)T + 1, 0), etiles((size_t)T, 0);
  for (int64_t t = 0; t < T; ++t) {
    eoff[(size_t)t] = (int64_t)ent.size();
    int64_t tl = 0;
    for (size_t i = 0; i < d.size(); ++i) {
      int64_t m0, c;
      plans[i].active(t, &m0, &c);
      if (c == 0) continue;
      ent.push_back(DiagEntry{(int)i, (int)m0, (int)c, (int)tl});
      tl += c * plans[i].G;
    }
    etiles[(size_t)t] = tl;
  }
  eoff[(size_t)T] = (int64_t)ent.size();
  if (tiles >= (size_t)INT32_MAX || otiles >= (size_t)INT32_MAX) return hipErrorInvalidValue;
  for (int64_t x : etiles)
    if (x >= INT32_MAX) return hipErrorInvalidValue;
  const size_t dbytes = align256(d.size() * sizeof(ProblemDesc));
  const size_t ebytes = align256(std::max<size_t>(1, ent.size()) * sizeof(DiagEntry));
  char* ws = nullptr;
  hipError_t err = ws_alloc((void**)&ws, dbytes + ebytes + qoff, st);
  if (err != hipSuccess) return err;
  for (size_t i = 0; i < d.size(); ++i) d[i].Qs = ws + dbytes + ebytes + qat[i];
  int dev = 0;
  (void)hipGetDevice(&dev);
  PinnedStaging& stage = PinnedStaging::for_device(dev);
  err = stage.upload(ws, d.data(), d.size() * sizeof(ProblemDesc), st);
  if (err == hipSuccess && !ent.empty())
    err = stage.upload(ws + dbytes, ent.data(), ent.size() * sizeof(DiagEntry), st);
  if (err != hipSuccess) {
    (void)ws_free(ws, st);
    return err;
  }
  const ProblemDesc* dd = (const ProblemDesc*)ws;
  const DiagEntry* de = (const DiagEntry*)(ws + dbytes);
  const int count = (int)d.size();
  hipLaunchKernelGGL(k_to_rows_b<E>, dim3((unsigned)tiles), dim3(256), 0, st, dd, count);
  ProfScope prof(st, K, S);
  for (int64_t t = 0; t < T; ++t) {
    const int64_t ne = eoff[(size_t)t + 1] - eoff[(size_t)t];
    if (ne == 0) continue;
    prof.before(st);
    hipLaunchKernelGGL((k_diag_b<E, NB, K, OCC>), dim3((unsigned)etiles[(size_t)t]), dim3(64), 0,
                       st, dd, de + eoff[(size_t)t], (int)ne, (int)t, opt.xcd);
    prof.after(st);
  }
  prof.end();
  hipLaunchKernelGGL(k_from_rows_b<E>, dim3((unsigned)otiles), dim3(256), 0, st, dd, count);
  err = hipGetLastError();
  const hipError_t e2 = ws_free(ws, st);
  return err != hipSuccess ? err : e2;
}

template <typename E, int NB, int K>
size_t diag_workspace(int64_t n, int64_t nev) {
  return DiagPlan(n, nev, NB, K, 1).template qbytes<E>();
}

}  // namespace ehh
