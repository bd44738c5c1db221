// HIP kernels (gfx950) of the tridiagonal->band eigenvector back-transformation
//
//     Q <- H(0,0) H(0,1) ... H(n-2, J-1) Q,      H(s,j) = I - tau v v^H,
//
// the two-stage solver's first back-transformation (Kus et al., Sec. 2; the
// compute-heavy part of the back-transformation singled out in Sec. 3.1).
//
// Stripe path (the fast one)
// --------------------------
// 1. Q (column major) is copied into a row-major workspace Qt whose rows hold
//    ldt = 64*G columns (G = ceil(nev/64) stripes) and which has zero rows
//    past n, enough for the deepest window.  A wave64 lane owns one column,
//    so a row of a 64-column stripe is one 512-byte coalesced access, and no
//    load or store needs a bounds check.
// 2. Work is split into tasks (stripe c, sweep block m): block m holds the K
//    consecutive sweeps [mK, mK+K-1].  A task slides a window of W = NB+K-1
//    rows of its stripe down the matrix, one chase step j = 0, 1, ... at a
//    time; at each step it applies the K reflectors (s, j) of its block,
//    largest s first, to the W rows held in VGPRs, writes the NB rows that
//    are final for this block and reads NB new ones.  Reflector values are
//    wave-uniform and come through scalar loads (SGPR operands of the FMAs).
//    Per lane and step: 2*NB*K FMAs per 2*NB row transfers.
// 3. Order.  Blocks of one stripe must run from the top (largest sweeps) down,
//    but only row by row: two reflectors (a, j), (c, j') with a > c share rows
//    only if a - c >= NB*(j'-j-1)+1, so block m at step j only needs block
//    m+1 to have finished its step j.  Each task publishes, after every step,
//    the row below which its stripe is final (release, agent scope); the task
//    of the next block waits on that value (acquire) before loading rows.
//    The result equals strict reverse generation order up to the rounding of
//    the dot products.
// 4. Scheduling.  A persistent grid takes tickets from an atomic counter in
//    dependency order (blocks descending, then stripes), so the task a wave
//    waits on always holds an earlier ticket and is running or done: no
//    deadlock, and every wave exits when the tickets run out.  Each stripe
//    has up to ~(n/NB) tasks in flight at once, which fills the chip even for
//    small nev.
// 5. Qt is copied back into Q.
//
// Reference path: any nbw, one reflector at a time, column-major in place.
#include "hh_common.h"
#include "hh_dispatch.h"
#include "hh_dpp.h"

#include <type_traits>

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
  const int64_t r0 = (int64_t)blockIdx.x * 64, c0 = (int64_t)blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 64 x 4
  for (int cc = ty; cc < 64; cc += 4) {
    const int64_t r = r0 + tx, c = c0 + cc;
    tile[cc][tx] = (r < n && c < nev) ? Q[r + c * ldq] : Ops<E>::zero();
  }
  __syncthreads();
  E* __restrict__ dst = Qs + (int64_t)blockIdx.y * rows_pad * 64;
  for (int rr = ty; rr < 64; rr += 4) {
    const int64_t r = r0 + rr;
    if (r < rows_pad) dst[r * 64 + tx] = tile[tx][rr];
  }
}

template <typename E>
__global__ __launch_bounds__(256) void k_from_rows(const E* __restrict__ Qs, int64_t rows_pad,
                                                   E* __restrict__ Q, int64_t ldq, int64_t n,
                                                   int64_t nev) {
  __shared__ E tile[64][65];
  const int64_t r0 = (int64_t)blockIdx.x * 64, c0 = (int64_t)blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const E* __restrict__ src = Qs + (int64_t)blockIdx.y * rows_pad * 64;
  for (int rr = ty; rr < 64; rr += 4) {
    const int64_t r = r0 + rr;
    if (r < n) tile[rr][tx] = src[r * 64 + tx];
  }
  __syncthreads();
  for (int cc = ty; cc < 64; cc += 4) {
    const int64_t r = r0 + tx, c = c0 + cc;
    if (r < n && c < nev) Q[r + c * ldq] = tile[tx][cc];
  }
}

__global__ void k_zero_i32(int* __restrict__ p, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0;
}

// ---------------------------------------------------------------------------
// Wavefront stripe kernel.
//   Qs      stripe-major workspace, row r of stripe c at Qs + (c*rows_pad + r)*64
//   prog    G*M ints (zeroed): prog[c*M + m] = rows final after task (c, m)
//   ticket  one int (zeroed)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wave_ticket(int* ticket) {
  int t = 0;
  if (threadIdx.x == 0) t = atomicAdd(ticket, 1);
  return __builtin_amdgcn_readfirstlane(t);
}

__device__ __forceinline__ int load_progress(const int* p) {
  return __builtin_amdgcn_readfirstlane(
      __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

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

__device__ __forceinline__ int zero_after(double d) {
  int z;
  asm("s_mov_b32 %0, 0" : "=s"(z) : "v"(d));
  return z;
}
__device__ __forceinline__ int zero_after(float d) {
  int z;
  asm("s_mov_b32 %0, 0" : "=s"(z) : "v"(d));
  return z;
}
__device__ __forceinline__ int zero_after(z64 d) { return zero_after(d.re); }

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

// Compile-time loop o = N-1, N-2, ..., 0 (every body gets a constant o, so
// the window indices stay static without relying on the unroller's budget).
template <int N>
struct RevFor {
  template <typename F>
  static __device__ __forceinline__ void run(F&& f) {
    f(std::integral_constant<int, N - 1>{});
    RevFor<N - 1>::run(f);
  }
};
template <>
struct RevFor<0> {
  template <typename F>
  static __device__ __forceinline__ void run(F&&) {}
};

template <typename E, int NB, int K, int OCC>
__global__ __launch_bounds__(64, OCC) void k_wave(const E* __restrict__ hh,
                                                const E* __restrict__ hh2,
                                                const E* __restrict__ tau, E* __restrict__ Qs,
                                                int64_t rows_pad, int64_t n, int G, int M,
                                                int* __restrict__ prog, int* ticket) {
  using O = Ops<E>;
  constexpr int W = NB + K - 1;
  const int lane = threadIdx.x;
  const int64_t ctot = csum(n - 1, NB);
  const int ntask = G * M;
  E x[W];
  for (;;) {
    const int tk = wave_ticket(ticket);
    if (tk >= ntask) break;
    const int m = M - 1 - tk / G;
    const int c = tk - (tk / G) * G;
    // uniform base of the stripe; row r of the lane's column is bp[r*64 + lane]
    E* __restrict__ bp = Qs + (int64_t)c * rows_pad * 64;
    const int64_t s0 = (int64_t)m * K;
    const int64_t s1 = (s0 + K - 1 < n - 2) ? s0 + K - 1 : n - 2;
    const int64_t J0 = (n - 1 - s0 + NB - 1) / NB;
    const int* pred = (m + 1 < M) ? prog + (int64_t)c * M + m + 1 : nullptr;
    int* mine = prog + (int64_t)c * M + m;
    int known = pred ? 0 : INT32_MAX;  // rows known final w.r.t. earlier blocks
    for (int64_t j = 0; j < J0; ++j) {
      const int64_t row0 = s0 + 1 + j * NB;
      // rows [row0, row0 + W) must be final w.r.t. block m+1
      int64_t need = row0 + W;
      if (need > n) need = n;
      if (known < need) {
        int p = load_progress(pred);
        while (p < need) {
          __builtin_amdgcn_s_sleep(1);
          p = load_progress(pred);
        }
        known = p;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
      E* __restrict__ rp = bp + row0 * 64;  // uniform
      if (j == 0) {
#pragma unroll
        for (int i = 0; i < W; ++i) x[i] = rp[i * 64 + lane];
      } else {
#pragma unroll
        for (int i = 0; i < K - 1; ++i) x[i] = x[i + NB];
#pragma unroll
        for (int i = K - 1; i < W; ++i) x[i] = rp[i * 64 + lane];
      }
      // slot of reflector (s0+o, j), or slot 0 with tau = 0 if it does not exist
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
        apply_reflector<E, NB, W>(x, o, hh + su * NB, hh2 + su * NB,
                                  hh + (sn < 0 ? 0 : sn) * NB, t, cur);
        sl = sn;
      });
#pragma unroll
      for (int i = 0; i < NB; ++i) rp[i * 64 + lane] = x[i];
      if (j + 1 < J0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (lane == 0)
          __hip_atomic_store(mine, (int)(row0 + NB), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    const int64_t rowl = s0 + 1 + (J0 - 1) * NB;
    E* __restrict__ rl = bp + rowl * 64;
#pragma unroll
    for (int i = NB; i < W; ++i) rl[i * 64 + lane] = x[i];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (lane == 0) __hip_atomic_store(mine, INT32_MAX, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Compile-time loop i = 0, 1, ..., N-1.
template <int N, int I = 0>
struct FwdFor {
  template <typename F>
  static __device__ __forceinline__ void run(F&& f) {
    if constexpr (I < N) {
      f(std::integral_constant<int, I>{});
      FwdFor<N, I + 1>::run(f);
    }
  }
};

// ---------------------------------------------------------------------------
// fp64 wavefront stripe kernel with DPP-broadcast reflector operands.
// Same tasks, order, window and progress protocol as k_wave; the reflector
// v (NB values) lives in NG = NB/16 VGPR pairs, lane l holding v[16g + l%16]
// in pair g, and tau in a VGPR; both are loaded with vector loads one
// reflector ahead.  The dot product uses NG independent accumulators (one per
// 16-value segment).
// ---------------------------------------------------------------------------
template <int NB, int K, int OCC>
__global__ __launch_bounds__(64, OCC) void k_wave_dpp(const double* __restrict__ hh,
                                                      const double* __restrict__ tau,
                                                      double* __restrict__ Qs, int64_t rows_pad,
                                                      int64_t n, int G, int M,
                                                      int* __restrict__ prog, int* ticket) {
  static_assert(NB == 32 || NB == 64, "DPP kernel supports NB = 32, 64");
  constexpr int NG = NB / 16;
  constexpr int W = NB + K - 1;
  const int lane = threadIdx.x;
  const int l16 = lane & 15;
  const int64_t ctot = csum(n - 1, NB);
  const int ntask = G * M;
  double x[W];
  for (;;) {
    const int tk = wave_ticket(ticket);
    if (tk >= ntask) break;
    const int m = M - 1 - tk / G;
    const int c = tk - (tk / G) * G;
    double* __restrict__ bp = Qs + (int64_t)c * rows_pad * 64;
    const int64_t s0 = (int64_t)m * K;
    const int64_t s1 = (s0 + K - 1 < n - 2) ? s0 + K - 1 : n - 2;
    const int64_t J0 = (n - 1 - s0 + NB - 1) / NB;
    const int* pred = (m + 1 < M) ? prog + (int64_t)c * M + m + 1 : nullptr;
    int* mine = prog + (int64_t)c * M + m;
    int known = pred ? 0 : INT32_MAX;
    for (int64_t j = 0; j < J0; ++j) {
      const int64_t row0 = s0 + 1 + j * NB;
      int64_t need = row0 + W;
      if (need > n) need = n;
      if (known < need) {
        int p = load_progress(pred);
        while (p < need) {
          __builtin_amdgcn_s_sleep(1);
          p = load_progress(pred);
        }
        known = p;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
      double* __restrict__ rp = bp + row0 * 64;
      if (j == 0) {
#pragma unroll
        for (int i = 0; i < W; ++i) x[i] = rp[i * 64 + lane];
      } else {
#pragma unroll
        for (int i = 0; i < K - 1; ++i) x[i] = x[i + NB];
#pragma unroll
        for (int i = K - 1; i < W; ++i) x[i] = rp[i * 64 + lane];
      }
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
#pragma unroll
      for (int i = 0; i < NB; ++i) rp[i * 64 + lane] = x[i];
      if (j + 1 < J0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (lane == 0)
          __hip_atomic_store(mine, (int)(row0 + NB), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    const int64_t rowl = s0 + 1 + (J0 - 1) * NB;
    double* __restrict__ rl = bp + rowl * 64;
#pragma unroll
    for (int i = NB; i < W; ++i) rl[i * 64 + lane] = x[i];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (lane == 0) __hip_atomic_store(mine, INT32_MAX, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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

// Workspace geometry of the stripe path.
template <typename E, int NB, int K>
void wave_geom(int64_t n, int64_t nev, int64_t* rows_pad, int64_t* G, int64_t* M,
               size_t* qbytes, size_t* bytes) {
  *G = (nev + 63) / 64;
  *M = (n - 1 + K - 1) / K;
  // deepest row touched: s0 + 1 + (J0-1)*NB + W - 1 < n + NB + K
  *rows_pad = ((n + NB + K + 63) / 64) * 64;
  *qbytes = (((size_t)(*rows_pad) * (size_t)(*G) * 64 * sizeof(E) + 255) / 256) * 256;
  *bytes = *qbytes + ((size_t)(*G) * (size_t)(*M) + 64) * sizeof(int);
}

// Which kernel runs a (type, NB, K, OCC) variant: fp64 uses the DPP kernel.
template <typename E, int NB, int K, int OCC>
struct WaveKernel {
  static void launch(dim3 g, hipStream_t st, const E* hh, const E* tau, E* Qs, int64_t rows_pad,
                     int64_t n, int G, int M, int* prog, int* ticket) {
    hipLaunchKernelGGL((k_wave<E, NB, K, OCC>), g, dim3(64), 0, st, hh, hh, tau, Qs, rows_pad, n,
                       G, M, prog, ticket);
  }
};
template <int NB, int K, int OCC>
struct WaveKernel<double, NB, K, OCC> {
  static void launch(dim3 g, hipStream_t st, const double* hh, const double* tau, double* Qs,
                     int64_t rows_pad, int64_t n, int G, int M, int* prog, int* ticket) {
    hipLaunchKernelGGL((k_wave_dpp<NB, K, OCC>), g, dim3(64), 0, st, hh, tau, Qs, rows_pad, n, G,
                       M, prog, ticket);
  }
};

template <typename E, int NB, int K, int OCC>
hipError_t launch_wave(const void* hh, const void* tau, void* Q, int64_t ldq, int64_t n,
                       int64_t nev, hipStream_t st, int num_cu) {
  int64_t rows_pad, G, M;
  size_t qbytes, bytes;
  wave_geom<E, NB, K>(n, nev, &rows_pad, &G, &M, &qbytes, &bytes);
  if (G * M + 64 >= INT32_MAX || n + NB + K >= INT32_MAX) return hipErrorInvalidValue;
  void* ws = nullptr;
  hipError_t err = hipMallocAsync(&ws, bytes, st);
  if (err != hipSuccess) return err;
  E* Qs = (E*)ws;
  int* prog = (int*)((char*)ws + qbytes);
  int* ticket = prog + G * M;
  const int64_t nint = G * M + 64;
  hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)((nint + 255) / 256)), dim3(256), 0, st, prog,
                     nint);
  hipLaunchKernelGGL(k_to_rows<E>, dim3((unsigned)(rows_pad / 64), (unsigned)G), dim3(256), 0, st,
                     (const E*)Q, ldq, n, nev, Qs, rows_pad);
  const int64_t want = (int64_t)num_cu * 4 * OCC;
  const int64_t grid = (G * M < want) ? G * M : want;
  WaveKernel<E, NB, K, OCC>::launch(dim3((unsigned)grid), st, (const E*)hh, (const E*)tau, Qs,
                                    rows_pad, n, (int)G, (int)M, prog, ticket);
  hipLaunchKernelGGL(k_from_rows<E>, dim3((unsigned)((n + 63) / 64), (unsigned)G), dim3(256), 0,
                     st, (const E*)Qs, rows_pad, (E*)Q, ldq, n, nev);
  err = hipGetLastError();
  const hipError_t e2 = hipFreeAsync(ws, st);
  return err != hipSuccess ? err : e2;
}

#define EHH_WAVE(E, DT, NB, K, OCC) {DT, NB, K, OCC, &launch_wave<E, NB, K, OCC>}

const StripeEntry* stripe_table(int* size) {
  static const StripeEntry table[] = {
      EHH_WAVE(double, 0, 32, 8, 2),  EHH_WAVE(double, 0, 32, 16, 2),
      EHH_WAVE(double, 0, 32, 32, 2), EHH_WAVE(double, 0, 32, 48, 1),
      EHH_WAVE(double, 0, 64, 8, 2),  EHH_WAVE(double, 0, 64, 16, 2),
      EHH_WAVE(double, 0, 64, 24, 2), EHH_WAVE(double, 0, 64, 32, 2),
      EHH_WAVE(double, 0, 64, 40, 1), EHH_WAVE(double, 0, 64, 48, 1),
      EHH_WAVE(float, 1, 32, 16, 2),  EHH_WAVE(float, 1, 32, 32, 2),
      EHH_WAVE(float, 1, 64, 16, 2),  EHH_WAVE(float, 1, 64, 32, 1),
      EHH_WAVE(z64, 2, 32, 4, 2),     EHH_WAVE(z64, 2, 32, 8, 1),
      EHH_WAVE(z64, 2, 64, 2, 1),     EHH_WAVE(z64, 2, 64, 4, 1),
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
