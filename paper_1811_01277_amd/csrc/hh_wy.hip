// WY-aggregated MFMA path (real fp64 and fp32) of the tridiagonal->band
// eigenvector back-transformation  Q <- H(0,0) H(0,1) ... H(n-2, J-1) Q
// (Kus et al., Sec. 2 and Sec. 3.1).
//
// Same block/step structure and diagonal launch schedule as the stripe
// kernels: blocks of K sweeps slide a window of W = NB+K-1 rows down a stripe,
// one chase step j at a time, applying the block's K reflectors (s0+o, j),
// o = K-1 .. 0.  Here the K reflectors of a step are applied as K/16
// sub-groups of 16 in compact-WY form:
//
//   H(a) H(a+1) ... H(a+15) = I - V T V^T          (a = s0 + 16u)
//
// V (column i = reflector a+i, starting i rows below the sub-group's first
// row; NB+16 rows, zero outside its support) and T (16 x 16 upper triangular,
// forward recurrence T_ii = tau_i, T[0:i, i] = -tau_i T[0:i, 0:i] V[:,0:i]^T v_i)
// are built once per (block, step, sub-group) by a pre-pass, which stores
// -U = -V T^T and V.  Per stripe the apply is two matrix products on MFMA
// tiles:
//
//   W' = (-U)^T X        (16 x SW, contraction over NB+16 window rows)
//   X  = X + V W'        ((NB+16) x SW, contraction over 16 reflectors)
//
// X is the stripe's window (SW = 16 columns per wave), held in LDS at fixed
// rows (the k-1 carried rows move down once per step, so every LDS address is
// a lane base plus a constant); W' passes through LDS between the products.  Executed flops
// per counted flop: (NB+16)/NB (the parallelogram's all-zero corner tiles are
// not computed beyond one 16-row tile).
#include "hh_common.h"
#include "hh_dispatch.h"
#include "hh_sched.h"

namespace ehh {

typedef double wy_d4 __attribute__((ext_vector_type(4)));
typedef float wy_f4 __attribute__((ext_vector_type(4)));

// One 16x16x4 MFMA: D = A (16x4) B (4x16) + C.  Lane l supplies A[l%16][l/16]
// and B[l/16][l%16]; element r of lane l's result is D[row(l/16, r)][l%16],
// with rows interleaved over the four result registers for fp64
// (row = l/16 + 4r) and blocked for fp32 (row = 4(l/16) + r) -- both checked
// on the device.
template <typename E>
struct Mfma;
template <>
struct Mfma<double> {
  using V4 = wy_d4;
  static __device__ __forceinline__ V4 run(double a, double b, V4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int q, int r) { return q + 4 * r; }
};
template <>
struct Mfma<float> {
  using V4 = wy_f4;
  static __device__ __forceinline__ V4 run(float a, float b, V4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int q, int r) { return 4 * q + r; }
};

template <int NB, int K>
struct WyGeom {
  static_assert(NB == 32 || NB == 64, "WY path supports NB = 32, 64");
  static_assert(K % 16 == 0 && K >= 16, "K must be a multiple of 16");
  static_assert(NB + K <= 128, "window (NB + K rows with the spare) must fit 16 KB of LDS");
  static constexpr int SG = K / 16;        // sub-groups per step
  static constexpr int RP = NB + 16;       // rows of a sub-group's V and U
  static constexpr int KS = RP / 4;        // MFMA k-steps over those rows
  static constexpr int RT = RP / 16;       // 16-row tiles of the update
  static constexpr int REC = 2 * RP * 16;  // packed record: -U then V, row major
  static constexpr int SW = 16;            // columns per stripe (one wave)
};

// Pre-pass: build -U = -V T^T and V of sub-group u of (block m, step j),
// g = (m * Jmax + j) * SG + u; one 256-thread block.
template <typename E, int NB, int K>
__device__ __forceinline__ void wy_prep_group(const E* __restrict__ hh,
                                              const E* __restrict__ tau, int64_t n,
                                              int64_t Jmax, E* __restrict__ P, int64_t g) {
  using Gm = WyGeom<NB, K>;
  constexpr int RP = Gm::RP;
  __shared__ double V[RP][17];
  __shared__ double Gr[16][17];
  __shared__ double T[16][17];
  __shared__ double tv[16];
  const int u = (int)(g % Gm::SG);
  const int64_t mj = g / Gm::SG;
  const int64_t m = mj / Jmax, j = mj % Jmax;
  const int64_t s0 = m * K;
  if (j >= (n - 1 - s0 + NB - 1) / NB) return;  // never read
  const int tid = threadIdx.x;
  const int64_t ctot = csum(n - 1, NB);
  for (int e = tid; e < RP * 16; e += 256) {
    const int rho = e / 16, i = e % 16;
    const int64_t s = s0 + 16 * u + i;
    double v = 0.0;
    if (s <= n - 2 && j < (n - 1 - s + NB - 1) / NB) {
      const int64_t slot = ctot - csum(n - 1 - s, NB) + j;
      const int64_t r = s + 1 + j * NB;
      const int64_t L = (NB < n - r) ? NB : n - r;
      const int d = rho - i;
      if (d >= 0 && d < L) v = (double)hh[slot * NB + d];
      if (rho == 0) tv[i] = (double)tau[slot];
    } else if (rho == 0) {
      tv[i] = 0.0;
    }
    V[rho][i] = v;
  }
  __syncthreads();
  {  // Gram matrix V^T V
    const int a = tid / 16, b = tid % 16;
    double acc = 0.0;
    for (int rho = 0; rho < RP; ++rho) acc += V[rho][a] * V[rho][b];
    Gr[a][b] = acc;
    T[a][b] = 0.0;
  }
  __syncthreads();
  if (tid < 16) T[tid][tid] = tv[tid];
  __syncthreads();
  // forward recurrence, column i: T[0:i, i] = -tau_i T[0:i, 0:i] G[0:i, i]
  for (int i = 1; i < 16; ++i) {
    if (tid < i) {
      double acc = 0.0;
      for (int l = tid; l < i; ++l) acc += T[tid][l] * Gr[l][i];
      T[tid][i] = -tv[i] * acc;
    }
    __syncthreads();
  }
  E* __restrict__ rec = P + (((m * Jmax + j) * Gm::SG) + u) * (int64_t)Gm::REC;
  for (int e = tid; e < RP * 16; e += 256) {
    const int rho = e / 16, i = e % 16;
    double acc = 0.0;  // U[rho][i] = sum_l V[rho][l] T[i][l], l >= i
    for (int l = i; l < 16; ++l) acc += V[rho][l] * T[i][l];
    rec[e] = (E)(-acc);
    rec[RP * 16 + e] = (E)V[rho][i];
  }
}

template <typename E, int NB, int K>
__global__ __launch_bounds__(256) void k_wy_prep(const E* __restrict__ hh,
                                                 const E* __restrict__ tau, int64_t n,
                                                 int64_t Jmax, E* __restrict__ P) {
  wy_prep_group<E, NB, K>(hh, tau, n, Jmax, P, blockIdx.x);
}

template <typename E, int NB, int K>
__global__ __launch_bounds__(256) void k_wy_prep_b(const ProblemDesc* __restrict__ d, int count) {
  const int b = (int)blockIdx.x;
  const ProblemDesc& D = d[find_by<ProblemDesc, &ProblemDesc::ptile0>(d, count, b)];
  wy_prep_group<E, NB, K>((const E*)D.hh, (const E*)D.tau, D.n, D.Jmax, (E*)D.P, b - D.ptile0);
}

// Layout conversion between Q and 16-column stripes (element (r, 16c + l) at
// Qs[(c*rows_pad + r)*16 + l]), 64 x 64 tiles (row band rt, column band ct)
// through LDS, padding written as zeros.
template <typename E>
__device__ __forceinline__ void to_rows16_tile(const E* __restrict__ Q, int64_t ldq, int64_t n,
                                               int64_t nev, E* __restrict__ Qs, int64_t rows_pad,
                                               int64_t G, int64_t rt, int64_t ct,
                                               E (*tile)[65]) {
  const int64_t r0 = rt * 64, c0 = ct * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int cc = ty; cc < 64; cc += 4) {
    const int64_t r = r0 + tx, col = c0 + cc;
    tile[cc][tx] = (r < n && col < nev) ? Q[r + col * ldq] : (E)0;
  }
  __syncthreads();
  const int64_t col = c0 + tx, c = col / 16, l = col % 16;
  if (c >= G) return;
  E* __restrict__ dst = Qs + c * rows_pad * 16 + l;
  for (int rr = ty; rr < 64; rr += 4) dst[(r0 + rr) * 16] = tile[tx][rr];
}

template <typename E>
__device__ __forceinline__ void from_rows16_tile(const E* __restrict__ Qs, int64_t rows_pad,
                                                 E* __restrict__ Q, int64_t ldq, int64_t n,
                                                 int64_t nev, int64_t G, int64_t rt, int64_t ct,
                                                 E (*tile)[65]) {
  const int64_t r0 = rt * 64, c0 = ct * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  {
    const int64_t col = c0 + tx, c = col / 16, l = col % 16;
    for (int rr = ty; rr < 64; rr += 4) {
      const int64_t r = r0 + rr;
      if (r < n && c < G) tile[rr][tx] = Qs[(c * rows_pad + r) * 16 + l];
    }
  }
  __syncthreads();
  for (int cc = ty; cc < 64; cc += 4) {
    const int64_t r = r0 + tx, col = c0 + cc;
    if (r < n && col < nev) Q[r + col * ldq] = tile[tx][cc];
  }
}

template <typename E>
__global__ __launch_bounds__(256) void k_to_rows16(const E* __restrict__ Q, int64_t ldq,
                                                   int64_t n, int64_t nev, E* __restrict__ Qs,
                                                   int64_t rows_pad, int64_t G) {
  __shared__ E tile[64][65];
  to_rows16_tile<E>(Q, ldq, n, nev, Qs, rows_pad, G, blockIdx.x, blockIdx.y, tile);
}

template <typename E>
__global__ __launch_bounds__(256) void k_from_rows16(const E* __restrict__ Qs, int64_t rows_pad,
                                                     E* __restrict__ Q, int64_t ldq, int64_t n,
                                                     int64_t nev, int64_t G) {
  __shared__ E tile[64][65];
  from_rows16_tile<E>(Qs, rows_pad, Q, ldq, n, nev, G, blockIdx.x, blockIdx.y, tile);
}

template <typename E>
__global__ __launch_bounds__(256) void k_to_rows16_b(const ProblemDesc* __restrict__ d,
                                                     int count) {
  __shared__ E tile[64][65];
  const int t = (int)blockIdx.x;
  const ProblemDesc& D = d[find_by<ProblemDesc, &ProblemDesc::tile0>(d, count, t)];
  const int local = t - D.tile0;
  to_rows16_tile<E>((const E*)D.Q, D.ldq, D.n, D.nev, (E*)D.Qs, D.rows_pad, D.G, local / D.GT,
                    local % D.GT, tile);
}

template <typename E>
__global__ __launch_bounds__(256) void k_from_rows16_b(const ProblemDesc* __restrict__ d,
                                                       int count) {
  __shared__ E tile[64][65];
  const int t = (int)blockIdx.x;
  const ProblemDesc& D = d[find_by<ProblemDesc, &ProblemDesc::otile0>(d, count, t)];
  const int local = t - D.otile0;
  from_rows16_tile<E>((const E*)D.Qs, D.rows_pad, (E*)D.Q, D.ldq, D.n, D.nev, D.G,
                      local / D.GT, local % D.GT, tile);
}

// The stripe's window in LDS: rows 0 .. W-1 (window row i = stripe row
// row0 + i) and one spare row W kept at zero (the top sub-group's products
// cover one row past the window, against zero entries of U and V).  16
// values per row; lane l accesses column l%16 of row l/16 + 4i.

// global rows [a, b) of the window <-> LDS rows [a, b)
template <typename E, bool TO_LDS>
__device__ __forceinline__ void win_copy(E* __restrict__ g, E* __restrict__ win, int a, int b) {
  const int l = threadIdx.x;
  for (int r4 = a; r4 < b; r4 += 4) {
    const int r = r4 + (l >> 4);
    if (r < b) {
      E* gp = g + (int64_t)r * 16 + (l & 15);
      E* lp = win + r * 16 + (l & 15);
      if (TO_LDS)
        *lp = *gp;
      else
        *gp = *lp;
    }
  }
}

// The MFMA operands one lane needs from a packed sub-group record: the A
// fragments of W' = (-U)^T X (element 64 kk + l of the row-major -U) ...
template <typename E, int NB, int K>
struct WyA {
  using Gm = WyGeom<NB, K>;
  E a[Gm::KS];
  __device__ __forceinline__ void load(const E* __restrict__ rec) {
#pragma unroll
    for (int kk = 0; kk < Gm::KS; ++kk) a[kk] = rec[64 * kk + threadIdx.x];
  }
};
// ... and those of the update X += V W' (V[16 rt + l%16][4 kk + l/16]).
template <typename E, int NB, int K>
struct WyV {
  using Gm = WyGeom<NB, K>;
  E v[Gm::RT][4];
  __device__ __forceinline__ void load(const E* __restrict__ rec) {
    const int l = threadIdx.x;
    const E* __restrict__ vv = rec + Gm::RP * 16 + (l & 15) * 16 + (l >> 4);
#pragma unroll
    for (int rt = 0; rt < Gm::RT; ++rt)
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) v[rt][kk] = vv[rt * 256 + 4 * kk];
  }
};

// One sub-group u (16 reflectors starting at window row 16u) applied to the
// wave's 16 columns of the LDS window.  A: this sub-group's first-product
// fragments (loaded during the previous sub-group's update); its update
// operands are loaded here, before the first product; `next` (if not null) is
// the record whose first-product fragments go into an during the update.
template <typename E, int NB, int K, int u>
__device__ __forceinline__ void wy_subgroup(const WyA<E, NB, K>& A, const E* __restrict__ rec,
                                            const E* __restrict__ next, WyA<E, NB, K>& an,
                                            E* __restrict__ win, E* __restrict__ wbuf) {
  using Gm = WyGeom<NB, K>;
  using MF = Mfma<E>;
  using V4 = typename MF::V4;
  const int l = threadIdx.x;
  const int lq = l >> 4, lj = l & 15;
  E* __restrict__ x = win + (16 * u) * 16 + l;  // row 16u + l/16, column l%16
  WyV<E, NB, K> Vop;
  Vop.load(rec);
  // W' = (-U)^T X, B = X[4 kk + l/16][l%16]; two accumulator chains
  V4 acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
#pragma unroll
  for (int kk = 0; kk < Gm::KS; ++kk) {
    const E b = x[64 * kk];
    if (kk & 1)
      acc1 = MF::run(A.a[kk], b, acc1);
    else
      acc0 = MF::run(A.a[kk], b, acc0);
  }
  // W'[row(q, r)][col] -> wbuf, row major (reflector, column)
#pragma unroll
  for (int r = 0; r < 4; ++r) wbuf[MF::row(lq, r) * 16 + lj] = acc0[r] + acc1[r];
  __syncthreads();
  if (next) an.load(next);
  // X += V W': per 16-row tile rt, D = X[16 rt + row(q, r)][col],
  // A = V[16 rt + l%16][4 kk + l/16], B = W'[4 kk + l/16][l%16]; the row tiles
  // are independent accumulator chains, interleaved
  E bw[4];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) bw[kk] = wbuf[(4 * kk + lq) * 16 + lj];
  E* __restrict__ xd = win + (16 * u) * 16 + lj;
  V4 d[Gm::RT];
#pragma unroll
  for (int rt = 0; rt < Gm::RT; ++rt)
#pragma unroll
    for (int r = 0; r < 4; ++r) d[rt][r] = xd[(16 * rt + MF::row(lq, r)) * 16];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk)
#pragma unroll
    for (int rt = 0; rt < Gm::RT; ++rt) d[rt] = MF::run(Vop.v[rt][kk], bw[kk], d[rt]);
#pragma unroll
  for (int rt = 0; rt < Gm::RT; ++rt)
#pragma unroll
    for (int r = 0; r < 4; ++r) xd[(16 * rt + MF::row(lq, r)) * 16] = d[rt][r];
  __syncthreads();
}

// One tile: group q (chase steps [qS, min(qS+S, J0))) of block m on stripe c.
template <typename E, int NB, int K>
__device__ __forceinline__ void run_wy_tile(const E* __restrict__ P, int64_t Jmax,
                                            E* __restrict__ Qs, int64_t rows_pad, int64_t n,
                                            int64_t c, int64_t m, int64_t q, int64_t S,
                                            E* __restrict__ win, E* __restrict__ wbuf) {
  using Gm = WyGeom<NB, K>;
  constexpr int W = NB + K - 1;
  constexpr int SG = Gm::SG;
  const int l = threadIdx.x;
  E* __restrict__ bp = Qs + c * rows_pad * 16;
  const int64_t s0 = m * K;
  const int64_t J0 = (n - 1 - s0 + NB - 1) / NB;
  const int64_t j0 = q * S;
  const int64_t j1 = (j0 + S < J0) ? j0 + S : J0;
  auto rec_of = [&](int64_t j, int u) -> const E* {
    return P + (((m * Jmax + j) * SG) + u) * (int64_t)Gm::REC;
  };
  WyA<E, NB, K> A[2];
  A[0].load(rec_of(j0, SG - 1));
  if (l < 16) win[W * 16 + l] = (E)0;  // spare row
  win_copy<E, true>(bp + (s0 + 1 + j0 * NB) * 16, win, 0, W);
  for (int64_t j = j0; j < j1; ++j) {
    E* __restrict__ rp = bp + (s0 + 1 + j * NB) * 16;
    __syncthreads();
    const E* next_step = (j + 1 < j1) ? rec_of(j + 1, SG - 1) : nullptr;
    // sub-groups SG-1 .. 0; A[(SG-1-u) % 2] holds sub-group u's fragments
    RevFor<SG>::run([&](auto uc) {
      constexpr int u = decltype(uc)::value;
      constexpr int cur = (SG - 1 - u) & 1;
      const E* nx = (u > 0) ? rec_of(j, u - 1) : next_step;
      wy_subgroup<E, NB, K, u>(A[cur], rec_of(j, u), nx, A[cur ^ 1], win, wbuf);
    });
    // an odd sub-group count leaves the next step's first fragments in A[1]
    if constexpr ((SG & 1) == 1) A[0] = A[1];
    win_copy<E, false>(rp, win, 0, NB);  // rows final for this block
    if (j + 1 < j1) {
      // carried rows NB .. W-1 move to 0 .. K-2; the next NB rows follow
      E t[(K - 1 + 3) / 4];
#pragma unroll
      for (int i = 0; i < (K - 1 + 3) / 4; ++i) {
        const int r = 4 * i + (l >> 4);
        t[i] = (r < K - 1) ? win[(NB + r) * 16 + (l & 15)] : (E)0;
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < (K - 1 + 3) / 4; ++i) {
        const int r = 4 * i + (l >> 4);
        if (r < K - 1) win[r * 16 + (l & 15)] = t[i];
      }
      win_copy<E, true>(rp + NB * 16, win, K - 1, W);
    }
  }
  __syncthreads();
  // carried rows (or final after the block's last step)
  win_copy<E, false>(bp + (s0 + 1 + (j1 - 1) * NB) * 16, win, NB, W);
}

template <typename E, int NB, int K, int OCC>
__global__ __launch_bounds__(64, OCC) void k_wy(const E* __restrict__ P, int64_t Jmax,
                                                E* __restrict__ Qs, int64_t rows_pad, int64_t n,
                                                int c0, int G, int M, int t, int m0, int S,
                                                int xcd) {
  __shared__ E win[(NB + K) * 16];
  __shared__ E wbuf[256];
  const int b = tile_of((int)blockIdx.x, (int)gridDim.x, xcd);
  const int c = c0 + b % G;
  const int m = m0 + b / G;
  run_wy_tile<E, NB, K>(P, Jmax, Qs, rows_pad, n, c, m, t - (M - 1 - m), S, win, wbuf);
}

template <typename E, int NB, int K, int OCC>
__global__ __launch_bounds__(64, OCC) void k_wy_b(const ProblemDesc* __restrict__ d,
                                                  const DiagEntry* __restrict__ e, int ecount,
                                                  int t, int xcd) {
  __shared__ E win[(NB + K) * 16];
  __shared__ E wbuf[256];
  const int b = tile_of((int)blockIdx.x, (int)gridDim.x, xcd);
  const DiagEntry& E0 = e[find_by<DiagEntry, &DiagEntry::tile0>(e, ecount, b)];
  const ProblemDesc& D = d[E0.p];
  const int local = b - E0.tile0;
  const int m = E0.m0 + local / D.G;
  run_wy_tile<E, NB, K>((const E*)D.P, D.Jmax, (E*)D.Qs, D.rows_pad, D.n, local % D.G, m,
                        t - (D.M - 1 - m), D.S, win, wbuf);
}

template <typename E, int NB, int K>
size_t wy_pbytes(int64_t M, int64_t Jmax) {
  using Gm = WyGeom<NB, K>;
  return align256((size_t)M * (size_t)Jmax * Gm::SG * Gm::REC * sizeof(E));
}

template <typename E, int NB, int K, int OCC>
hipError_t launch_wy(const void* hh, const void* tau, void* Q, int64_t ldq, int64_t n,
                     int64_t nev, TileOpts opt, hipStream_t st, int num_cu) {
  using Gm = WyGeom<NB, K>;
  static const int64_t slots = wave_slots(k_wy<E, NB, K, OCC>, num_cu);
  const int64_t S = opt.steps > 0 ? opt.steps : choose_steps(n, nev, NB, K, slots, Gm::SW);
  const DiagPlan pl(n, nev, NB, K, S, Gm::SW);
  const int64_t Jmax = (n - 1 + NB - 1) / NB;
  if (pl.G * pl.M >= INT32_MAX || pl.M * Jmax * Gm::SG >= INT32_MAX || n + NB + K >= INT32_MAX)
    return hipErrorInvalidValue;
  const size_t pbytes = wy_pbytes<E, NB, K>(pl.M, Jmax);
  char* ws = nullptr;
  hipError_t err = ws_alloc((void**)&ws, pbytes + pl.template qbytes<E>(), st);
  if (err != hipSuccess) return err;
  E* Pk = (E*)ws;
  E* Qs = (E*)(ws + pbytes);
  const unsigned gt = (unsigned)((nev + 63) / 64);
  hipLaunchKernelGGL((k_wy_prep<E, NB, K>), dim3((unsigned)(pl.M * Jmax * Gm::SG)), dim3(256), 0,
                     st, (const E*)hh, (const E*)tau, n, Jmax, Pk);
  hipLaunchKernelGGL(k_to_rows16<E>, dim3((unsigned)(pl.rows_pad / 64), gt), dim3(256), 0, st,
                     (const E*)Q, ldq, n, nev, Qs, pl.rows_pad, pl.G);
  const int ns = (int)std::max<int64_t>(1, std::min<int64_t>(opt.streams, pl.G));
  ProfScope prof(st, K, S, ns);
  {
    StreamFork fork(st, ns);
    if (fork.error() != hipSuccess) {
      (void)hipFreeAsync(ws, st);
      return fork.error();
    }
    for (int64_t t = 0; t < pl.T; ++t) {
      int64_t m0, cnt;
      pl.active(t, &m0, &cnt);
      if (cnt == 0) continue;
      for (int i = 0; i < ns; ++i) {
        const int64_t c_lo = pl.G * i / ns, gs = pl.G * (i + 1) / ns - c_lo;
        prof.before(fork.stream(i));
        hipLaunchKernelGGL((k_wy<E, NB, K, OCC>), dim3((unsigned)(cnt * gs)), dim3(64), 0,
                           fork.stream(i), (const E*)Pk, Jmax, Qs, pl.rows_pad, n, (int)c_lo,
                           (int)gs, (int)pl.M, (int)t, (int)m0, (int)S, opt.xcd);
        prof.after(fork.stream(i));
      }
    }
    err = fork.join();
  }
  prof.end();
  if (err != hipSuccess) {
    (void)hipFreeAsync(ws, st);
    return err;
  }
  hipLaunchKernelGGL(k_from_rows16<E>, dim3((unsigned)((n + 63) / 64), gt), dim3(256), 0, st,
                     (const E*)Qs, pl.rows_pad, (E*)Q, ldq, n, nev, pl.G);
  err = hipGetLastError();
  const hipError_t e2 = hipFreeAsync(ws, st);
  return err != hipSuccess ? err : e2;
}

// Batched: problems idx[0..cnt) of probs (element type E, semi-bandwidth NB,
// validated by the caller); all problems' diagonal schedules side by side.
template <typename E, int NB, int K, int OCC>
hipError_t launch_wy_batched(const elpa_hh_problem* probs, const int64_t* idx, int64_t cnt,
                             TileOpts opt, hipStream_t st, int num_cu) {
  using Gm = WyGeom<NB, K>;
  const int64_t S = opt.steps;
  static const int64_t slots = wave_slots(k_wy_b<E, NB, K, OCC>, num_cu);
  std::vector<ProblemDesc> d;
  std::vector<DiagPlan> plans;
  int64_t total_cols = 0;
  for (int64_t i = 0; i < cnt; ++i) {
    const elpa_hh_problem& p = probs[idx[i]];
    if (p.n > 1 && p.nev > 0) total_cols += p.nev;
  }
  for (int64_t i = 0; i < cnt; ++i) {
    const elpa_hh_problem& p = probs[idx[i]];
    if (p.n <= 1 || p.nev == 0) continue;
    const int64_t s = S > 0 ? S : choose_steps(p.n, total_cols, NB, K, slots, Gm::SW);
    plans.emplace_back(p.n, p.nev, NB, K, s, Gm::SW);
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
  size_t off = 0, tiles = 0, otiles = 0, ptiles = 0;
  int64_t T = 0;
  std::vector<size_t> pat(d.size()), qat(d.size());
  for (size_t i = 0; i < d.size(); ++i) {
    const DiagPlan& pl = plans[i];
    const int64_t Jmax = (pl.n - 1 + NB - 1) / NB;
    d[i].G = (int)pl.G;
    d[i].GT = (int)((pl.nev + 63) / 64);
    d[i].M = (int)pl.M;
    d[i].S = (int)pl.S;
    d[i].rows_pad = pl.rows_pad;
    d[i].Jmax = Jmax;
    d[i].tile0 = (int)tiles;
    d[i].otile0 = (int)otiles;
    d[i].ptile0 = (int)ptiles;
    tiles += (size_t)(pl.rows_pad / 64 * d[i].GT);
    otiles += (size_t)((pl.n + 63) / 64 * d[i].GT);
    ptiles += (size_t)(pl.M * Jmax * Gm::SG);
    pat[i] = off;
    off += wy_pbytes<E, NB, K>(pl.M, Jmax);
    qat[i] = off;
    off += pl.template qbytes<E>();
    T = std::max(T, pl.T);
  }
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
  if (tiles >= (size_t)INT32_MAX || otiles >= (size_t)INT32_MAX || ptiles >= (size_t)INT32_MAX)
    return hipErrorInvalidValue;
  for (int64_t x : etiles)
    if (x >= INT32_MAX) return hipErrorInvalidValue;
  const size_t dbytes = align256(d.size() * sizeof(ProblemDesc));
  const size_t ebytes = align256(std::max<size_t>(1, ent.size()) * sizeof(DiagEntry));
  char* ws = nullptr;
  hipError_t err = ws_alloc((void**)&ws, dbytes + ebytes + off, st);
  if (err != hipSuccess) return err;
  for (size_t i = 0; i < d.size(); ++i) {
    d[i].P = ws + dbytes + ebytes + pat[i];
    d[i].Qs = ws + dbytes + ebytes + qat[i];
  }
  int dev = 0;
  (void)hipGetDevice(&dev);
  PinnedStaging& stage = PinnedStaging::for_device(dev);
  err = stage.upload(ws, d.data(), d.size() * sizeof(ProblemDesc), st);
  if (err == hipSuccess && !ent.empty())
    err = stage.upload(ws + dbytes, ent.data(), ent.size() * sizeof(DiagEntry), st);
  if (err != hipSuccess) {
    (void)hipFreeAsync(ws, st);
    return err;
  }
  const ProblemDesc* dd = (const ProblemDesc*)ws;
  const DiagEntry* de = (const DiagEntry*)(ws + dbytes);
  const int count = (int)d.size();
  hipLaunchKernelGGL((k_wy_prep_b<E, NB, K>), dim3((unsigned)ptiles), dim3(256), 0, st, dd, count);
  hipLaunchKernelGGL(k_to_rows16_b<E>, dim3((unsigned)tiles), dim3(256), 0, st, dd, count);
  ProfScope prof(st, K, S);
  for (int64_t t = 0; t < T; ++t) {
    const int64_t ne = eoff[(size_t)t + 1] - eoff[(size_t)t];
    if (ne == 0) continue;
    prof.before(st);
    hipLaunchKernelGGL((k_wy_b<E, NB, K, OCC>), dim3((unsigned)etiles[(size_t)t]), dim3(64), 0, st,
                       dd, de + eoff[(size_t)t], (int)ne, (int)t, opt.xcd);
    prof.after(st);
  }
  prof.end();
  hipLaunchKernelGGL(k_from_rows16_b<E>, dim3((unsigned)otiles), dim3(256), 0, st, dd, count);
  err = hipGetLastError();
  const hipError_t e2 = hipFreeAsync(ws, st);
  return err != hipSuccess ? err : e2;
}

template <typename E, int NB, int K>
size_t wy_workspace(int64_t n, int64_t nev) {
  const DiagPlan pl(n, nev, NB, K, 1, WyGeom<NB, K>::SW);
  return wy_pbytes<E, NB, K>(pl.M, (n - 1 + NB - 1) / NB) + pl.template qbytes<E>();
}

#define EHH_WY(E, DT, NB, K, OCC) \
  {ELPA_PATH_WY,     DT, NB, K, OCC, &launch_wy<E, NB, K, OCC>, &launch_wy_batched<E, NB, K, OCC>, \
   &wy_workspace<E, NB, K>}

const StripeEntry* wy_table(int* size) {
  static const StripeEntry table[] = {
      EHH_WY(double, 0, 64, 32, 2), EHH_WY(double, 0, 64, 48, 2), EHH_WY(double, 0, 64, 64, 2),
      EHH_WY(double, 0, 32, 32, 2), EHH_WY(double, 0, 32, 64, 2), EHH_WY(double, 0, 32, 96, 2),
      EHH_WY(float, 1, 64, 32, 2),  EHH_WY(float, 1, 64, 64, 2),  EHH_WY(float, 1, 32, 64, 2),
      EHH_WY(float, 1, 32, 96, 2),
  };
  *size = (int)(sizeof(table) / sizeof(table[0]));
  return table;
}

}  // namespace ehh
