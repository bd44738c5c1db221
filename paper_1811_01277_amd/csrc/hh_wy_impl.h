// Compact-WY MFMA path (real fp64, real fp32, complex fp64) of the
// tridiagonal->band eigenvector back-transformation
//
//     Q <- H(0,0) H(0,1) ... H(n-2, J-1) Q       (Kus et al., Sec. 2, Sec. 3.1)
//
// Same block/step order and diagonal launch schedule as the stripe kernels:
// blocks of K sweeps slide a window of NB+K rows down a stripe of Q, one chase
// step j at a time, applying the block's reflectors (s0+o, j), o = K-1 .. 0.
// Here the K reflectors of a step are applied as K/16 sub-groups of 16 in
// compact-WY form,
//
//     H(a) H(a+1) ... H(a+15) = I - V T V^H,        a = s0 + 16u,
//
// with V (NB+16 rows: column i is reflector a+i starting i rows below the
// sub-group's first window row 16u, zero outside its support) and T (16 x 16
// upper triangular, the forward recurrence T_ii = tau_i,
// T[0:i, i] = -tau_i T[0:i, 0:i] V[:, 0:i]^H v_i) built once per (block, step,
// sub-group) by a pre-pass.  With U = V T^H the application is
//
//     W' = (-U)^H X        (16 x SW, contraction over the NB+16 rows)
//     X  = X + V W'        ((NB+16) x SW, contraction over the 16 reflectors)
//
// on 16x16x4 MFMA tiles.  Complex values are planar: each complex product is
// four real MFMA chains.
//
// Registers, not LDS.  A wave owns a stripe of SW = 16 T columns; its window
// is held as (NB+K)/16 x T tiles of 16 x 16 in the MFMA result layout (lane l,
// quad q = l/16, holds column l%16 and rows row(q, r), r = 0..3).  The
// contraction index of MFMA k-step kk is mapped to row(q, kk) of a 16-row
// tile, so a result tile is directly the B operand of the next product: the
// window feeds W' = (-U)^H X and W' feeds the update without any data
// movement.  The pre-pass stores each sub-group's A fragments of (-U)^H and of
// V in exactly that mapping, one 64-lane vector per fragment, so every operand
// load is one coalesced 512-byte (fp64) access and each fragment feeds T
// MFMAs (one per column tile).  The next sub-group's (-U)^H fragments load
// during the current update, the current V fragments during the first
// product.
//
// Executed flops per counted flop: (NB+16)/NB (the sub-group's parallelogram
// padded to whole 16-row tiles).
#pragma once

#include "hh_common.h"
#include "hh_dispatch.h"
#include "hh_layout.h"
#include "hh_sched.h"

namespace ehh {

typedef double wy_d4 __attribute__((ext_vector_type(4)));
typedef float wy_f4 __attribute__((ext_vector_type(4)));

// Element traits: R = real scalar of records and MFMA operands, PL = planes.
template <typename E>
struct WyElem;
template <>
struct WyElem<double> {
  using R = double;
  using V4 = wy_d4;
  static constexpr int PL = 1;
  static constexpr bool kInterleaved = true;
};
template <>
struct WyElem<float> {
  using R = float;
  using V4 = wy_f4;
  static constexpr int PL = 1;
  static constexpr bool kInterleaved = false;
};
template <>
struct WyElem<z64> {
  using R = double;
  using V4 = wy_d4;
  static constexpr int PL = 2;
  static constexpr bool kInterleaved = true;
};

__device__ __forceinline__ wy_d4 wy_mfma(double a, double b, wy_d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ wy_f4 wy_mfma(float a, float b, wy_f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Row of a 16-row tile in result register r of lane quad q: interleaved
// (q + 4r) for the fp64 MFMA, blocked (4q + r) for fp32 (both layouts
// checked on the device).
template <bool kInterleaved>
__host__ __device__ constexpr int wy_row(int q, int r) {
  return kInterleaved ? q + 4 * r : 4 * q + r;
}

template <int NB, int K>
struct WyGeom {
  static_assert(NB == 32 || NB == 64, "WY path supports NB = 32, 64");
  static_assert(K % 16 == 0 && K >= 16, "K must be a multiple of 16");
  static constexpr int SG = K / 16;          // sub-groups per step
  static constexpr int RT = NB / 16 + 1;     // 16-row tiles a sub-group touches
  static constexpr int RTW = (NB + K) / 16;  // 16-row tiles of the window
  static constexpr int NF = 4 * RT;          // MFMA fragments per operand and plane
  static constexpr int RP = NB + 16;         // rows of a sub-group's V
};

template <typename E, int NB, int K>
struct WyRec {
  using G = WyGeom<NB, K>;
  static constexpr int PL = WyElem<E>::PL;
  // planes of 64-lane fragments: (-U)^H re [, im], then V re [, im]
  static constexpr int REC = 2 * PL * G::NF * 64;
};

// ---------------------------------------------------------------------------
// pre-pass: V, T and the operand fragments of sub-group u of (block m, step j)
// ---------------------------------------------------------------------------
template <typename E>
__device__ __forceinline__ void wy_get(const E& x, double& re, double& im);
template <>
__device__ __forceinline__ void wy_get<double>(const double& x, double& re, double& im) {
  re = x;
  im = 0.0;
}
template <>
__device__ __forceinline__ void wy_get<float>(const float& x, double& re, double& im) {
  re = (double)x;
  im = 0.0;
}
template <>
__device__ __forceinline__ void wy_get<z64>(const z64& x, double& re, double& im) {
  re = x.re;
  im = x.im;
}

// One 256-thread block; the block of step 0, sub-group 0 also writes Bt[m],
// the first step record of block m.
template <typename E, int NB, int K>
__device__ __forceinline__ void wy_prep_group(const E* __restrict__ hh, const E* __restrict__ tau,
                                              int64_t n, int64_t m, int64_t j, int u,
                                              typename WyElem<E>::R* __restrict__ P,
                                              int64_t* __restrict__ Bt) {
  using Gm = WyGeom<NB, K>;
  using R = typename WyElem<E>::R;
  constexpr int RP = Gm::RP, NF = Gm::NF, PL = WyElem<E>::PL;
  constexpr bool CPLX = PL == 2;
  __shared__ double Vr[RP][17], Vi[RP][17];
  __shared__ double Gr[16][17], Gi[16][17];
  __shared__ double Tr[16][17], Ti[16][17];
  __shared__ double tr_[16], ti_[16];
  __shared__ int64_t slot_[16];  // slot of reflector i, -1 if it does not exist
  __shared__ int len_[16];       // its length L
  __shared__ int64_t mb_;        // the block's first step record
  const int64_t s0 = m * K;
  if (j >= block_steps(n, NB, K, m)) return;  // no such step
  const int tid = threadIdx.x;
  // 64-bit integer divisions are emulated in many instructions: the block
  // base (a floor sum) and the slots are computed once, by one and sixteen
  // threads, not by every thread
  if (tid == 64) {
    mb_ = block_base(n, NB, K, m);
    if (j == 0 && u == 0) Bt[m] = mb_;
  }
  if (tid < 16) {  // the sub-group's 16 slots, once
    const int64_t s = s0 + 16 * u + tid;
    int64_t slot = -1;
    int L = 0;
    if (s <= n - 2 && j < (n - 1 - s + NB - 1) / NB) {
      slot = csum(n - 1, NB) - csum(n - 1 - s, NB) + j;
      const int64_t r = s + 1 + j * NB;
      L = (int)((NB < n - r) ? NB : n - r);
    }
    slot_[tid] = slot;
    len_[tid] = L;
    if (slot >= 0) {
      wy_get<E>(tau[slot], tr_[tid], ti_[tid]);
    } else {
      tr_[tid] = 0.0;
      ti_[tid] = 0.0;
    }
  }
  __syncthreads();
  // consecutive threads take consecutive entries of one slot (coalesced)
  for (int e = tid; e < RP * 16; e += 256) {
    const int i = e / RP, rho = e % RP;
    const int64_t slot = slot_[i];
    const int d = rho - i;
    double vr = 0.0, vi = 0.0;
    if (slot >= 0 && d >= 0 && d < len_[i]) wy_get<E>(hh[slot * NB + d], vr, vi);
    Vr[rho][i] = vr;
    Vi[rho][i] = vi;
  }
  __syncthreads();
  // (real data: the imaginary parts are zero and their terms are skipped)
  {  // Gram matrix G = V^H V
    const int a = tid / 16, b = tid % 16;
    double gr = 0.0, gi = 0.0;
    for (int rho = 0; rho < RP; ++rho) {
      // conj(V[rho][a]) V[rho][b]
      if constexpr (CPLX) {
        gr += Vr[rho][a] * Vr[rho][b] + Vi[rho][a] * Vi[rho][b];
        gi += Vr[rho][a] * Vi[rho][b] - Vi[rho][a] * Vr[rho][b];
      } else {
        gr += Vr[rho][a] * Vr[rho][b];
      }
    }
    Gr[a][b] = gr;
    Gi[a][b] = gi;
    Tr[a][b] = 0.0;
    Ti[a][b] = 0.0;
  }
  __syncthreads();
  // forward recurrence, column i: T[0:i, i] = -tau_i T[0:i, 0:i] G[0:i, i].
  // Entry (a, i) needs only row a of T (T[a][l] = 0 for l < a), so lane a
  // computes its whole row in column order, with no barrier in between.
  if (tid < 16) {
    Tr[tid][tid] = tr_[tid];
    Ti[tid][tid] = ti_[tid];
    for (int i = tid + 1; i < 16; ++i) {
      double ar = 0.0, ai = 0.0;
      for (int l = tid; l < i; ++l) {
        if constexpr (CPLX) {
          ar += Tr[tid][l] * Gr[l][i] - Ti[tid][l] * Gi[l][i];
          ai += Tr[tid][l] * Gi[l][i] + Ti[tid][l] * Gr[l][i];
        } else {
          ar += Tr[tid][l] * Gr[l][i];
        }
      }
      if constexpr (CPLX) {
        Tr[tid][i] = -(tr_[i] * ar - ti_[i] * ai);
        Ti[tid][i] = -(tr_[i] * ai + ti_[i] * ar);
      } else {
        Tr[tid][i] = -(tr_[i] * ar);
      }
    }
  }
  __syncthreads();
  R* __restrict__ rec = P + ((mb_ + j) * Gm::SG + u) * (int64_t)WyRec<E, NB, K>::REC;
  for (int e = tid; e < NF * 64; e += 256) {
    const int f = e / 64, lane = e % 64;
    const int rt = f / 4, kk = f % 4;
    const int q = lane >> 4, c = lane & 15;
    const int k = wy_row<WyElem<E>::kInterleaved>(q, kk);
    // (-U)^H [c][16 rt + k] = -conj(U[16 rt + k][c]),
    // U[rho][c] = sum_{l >= c} V[rho][l] conj(T[c][l])
    const int rho = 16 * rt + k;
    double ur = 0.0, ui = 0.0;
    for (int l = c; l < 16; ++l) {
      if constexpr (CPLX) {
        ur += Vr[rho][l] * Tr[c][l] + Vi[rho][l] * Ti[c][l];
        ui += Vi[rho][l] * Tr[c][l] - Vr[rho][l] * Ti[c][l];
      } else {
        ur += Vr[rho][l] * Tr[c][l];
      }
    }
    rec[(0 * NF + f) * 64 + lane] = (R)(-ur);
    if constexpr (CPLX) rec[(1 * NF + f) * 64 + lane] = (R)ui;
    // V[16 rt + c][k]
    rec[(PL * NF + f) * 64 + lane] = (R)Vr[16 * rt + c][k];
    if constexpr (CPLX) rec[((PL + 1) * NF + f) * 64 + lane] = (R)Vi[16 * rt + c][k];
  }
}

template <typename E, int NB, int K>
__global__ __launch_bounds__(256) void k_wy_prep(const E* __restrict__ hh,
                                                 const E* __restrict__ tau, int64_t n,
                                                 int64_t Jmax, typename WyElem<E>::R* __restrict__ P,
                                                 int64_t* __restrict__ Bt) {
  using Gm = WyGeom<NB, K>;
  const int64_t g = blockIdx.x;
  const int u = (int)(g % Gm::SG);
  const int64_t mj = g / Gm::SG;
  wy_prep_group<E, NB, K>(hh, tau, n, mj / Jmax, mj % Jmax, u, P, Bt);
}

template <typename E, int NB, int K>
__global__ __launch_bounds__(256) void k_wy_prep_b(const ProblemDesc* __restrict__ d, int count) {
  using Gm = WyGeom<NB, K>;
  const int b = (int)blockIdx.x;
  const ProblemDesc& D = d[find_by<ProblemDesc, &ProblemDesc::ptile0>(d, count, b)];
  const int64_t g = b - D.ptile0;
  const int u = (int)(g % Gm::SG);
  const int64_t mj = g / Gm::SG;
  wy_prep_group<E, NB, K>((const E*)D.hh, (const E*)D.tau, D.n, mj / D.Jmax, mj % D.Jmax, u,
                          (typename WyElem<E>::R*)D.P, (int64_t*)D.Bt);
}

// ---------------------------------------------------------------------------
// apply
// ---------------------------------------------------------------------------
template <typename E, int NB, int K>
struct WyA {  // (-U)^H fragments of one sub-group
  using R = typename WyElem<E>::R;
  static constexpr int PL = WyElem<E>::PL, NF = WyGeom<NB, K>::NF;
  R a[PL][NF];
  __device__ __forceinline__ void load(const R* __restrict__ rec) {
#pragma unroll
    for (int p = 0; p < PL; ++p)
#pragma unroll
      for (int f = 0; f < NF; ++f) a[p][f] = rec[(p * NF + f) * 64 + threadIdx.x];
  }
};
template <typename E, int NB, int K>
struct WyV {  // V fragments of one sub-group
  using R = typename WyElem<E>::R;
  static constexpr int PL = WyElem<E>::PL, NF = WyGeom<NB, K>::NF;
  R v[PL][NF];
  __device__ __forceinline__ void load(const R* __restrict__ rec) {
#pragma unroll
    for (int p = 0; p < PL; ++p)
#pragma unroll
      for (int f = 0; f < NF; ++f) v[p][f] = rec[((PL + p) * NF + f) * 64 + threadIdx.x];
  }
};

// The stripe window: x[p][tr][t] is 16-row tile tr, column tile t of plane p.
template <typename E, int NB, int K, int T>
struct WyWin {
  using V4 = typename WyElem<E>::V4;
  static constexpr int PL = WyElem<E>::PL, RTW = WyGeom<NB, K>::RTW;
  V4 x[PL][RTW][T];
};

template <typename E>
__device__ __forceinline__ void wy_split(const E& v, typename WyElem<E>::R (&o)[WyElem<E>::PL]);
template <>
__device__ __forceinline__ void wy_split<double>(const double& v, double (&o)[1]) {
  o[0] = v;
}
template <>
__device__ __forceinline__ void wy_split<float>(const float& v, float (&o)[1]) {
  o[0] = v;
}
template <>
__device__ __forceinline__ void wy_split<z64>(const z64& v, double (&o)[2]) {
  o[0] = v.re;
  o[1] = v.im;
}
template <typename E>
__device__ __forceinline__ E wy_join(const typename WyElem<E>::R (&o)[WyElem<E>::PL]);
template <>
__device__ __forceinline__ double wy_join<double>(const double (&o)[1]) {
  return o[0];
}
template <>
__device__ __forceinline__ float wy_join<float>(const float (&o)[1]) {
  return o[0];
}
template <>
__device__ __forceinline__ z64 wy_join<z64>(const double (&o)[2]) {
  return z64{o[0], o[1]};
}

// window tile tr <-> stripe rows row0 + 16 tr + row(q, r), columns 16 t + l%16
template <typename E, int NB, int K, int T, int SW>
__device__ __forceinline__ void wy_load_tile(WyWin<E, NB, K, T>& w, int tr,
                                             const E* __restrict__ rp) {
  using R = typename WyElem<E>::R;
  constexpr int PL = WyElem<E>::PL;
  const int l = threadIdx.x, q = l >> 4, cl = l & 15;
#pragma unroll
  for (int t = 0; t < T; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const E v = rp[(16 * tr + wy_row<WyElem<E>::kInterleaved>(q, r)) * SW + 16 * t + cl];
      R o[PL];
      wy_split<E>(v, o);
#pragma unroll
      for (int p = 0; p < PL; ++p) w.x[p][tr][t][r] = o[p];
    }
}

// skip_last: leave the tile's last row (row 15: quad 3, register 3) unwritten
template <typename E, int NB, int K, int T, int SW>
__device__ __forceinline__ void wy_store_tile(const WyWin<E, NB, K, T>& w, int tr,
                                              E* __restrict__ rp, bool skip_last) {
  using R = typename WyElem<E>::R;
  constexpr int PL = WyElem<E>::PL;
  const int l = threadIdx.x, q = l >> 4, cl = l & 15;
#pragma unroll
  for (int t = 0; t < T; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (skip_last && r == 3 && q == 3) continue;
      R o[PL];
#pragma unroll
      for (int p = 0; p < PL; ++p) o[p] = w.x[p][tr][t][r];
      rp[(16 * tr + wy_row<WyElem<E>::kInterleaved>(q, r)) * SW + 16 * t + cl] = wy_join<E>(o);
    }
}

// Sub-group u applied to the window: W' = (-U)^H X over tiles u .. u+RT-1,
// then X += V W' on the same tiles.  A: this sub-group's (-U)^H fragments;
// its V fragments are loaded here; `next` (if not null) is the record whose
// (-U)^H fragments go into An during the update.
// With VP, Vin holds this sub-group's V fragments (loaded a sub-group ahead)
// and Vn receives the next sub-group's during the first product; without VP
// they are loaded here.
template <typename E, int NB, int K, int T, int u, bool VP>
__device__ __forceinline__ void wy_subgroup(WyWin<E, NB, K, T>& w, const WyA<E, NB, K>& A,
                                            const typename WyElem<E>::R* __restrict__ rec,
                                            const typename WyElem<E>::R* __restrict__ next,
                                            WyA<E, NB, K>& An, const WyV<E, NB, K>& Vin,
                                            WyV<E, NB, K>& Vn) {
  using Gm = WyGeom<NB, K>;
  using V4 = typename WyElem<E>::V4;
  constexpr int PL = WyElem<E>::PL, RT = Gm::RT;
  WyV<E, NB, K> Vown;
  if constexpr (VP) {
    if (next) Vn.load(next);
  } else {
    Vown.load(rec);
  }
  const WyV<E, NB, K>& Vop = VP ? Vin : Vown;
  V4 wr[T], wi[T];
  if constexpr (PL == 1) {
    V4 a0[T], a1[T];
#pragma unroll
    for (int t = 0; t < T; ++t) a0[t] = a1[t] = V4{0, 0, 0, 0};
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
#pragma unroll
        for (int t = 0; t < T; ++t) {
          if (kk & 1)
            a1[t] = wy_mfma(A.a[0][4 * rt + kk], w.x[0][u + rt][t][kk], a1[t]);
          else
            a0[t] = wy_mfma(A.a[0][4 * rt + kk], w.x[0][u + rt][t][kk], a0[t]);
        }
#pragma unroll
    for (int t = 0; t < T; ++t) wr[t] = a0[t] + a1[t];
  } else {
    // W' = A X, A = Ar + i Ai:  re = Ar Xr - Ai Xi,  im = Ar Xi + Ai Xr
    V4 rr[T], ii[T], ri[T], ir[T];
#pragma unroll
    for (int t = 0; t < T; ++t) rr[t] = ii[t] = ri[t] = ir[t] = V4{0, 0, 0, 0};
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
#pragma unroll
        for (int t = 0; t < T; ++t) {
          const int f = 4 * rt + kk;
          rr[t] = wy_mfma(A.a[0][f], w.x[0][u + rt][t][kk], rr[t]);
          ii[t] = wy_mfma(A.a[1][f], w.x[1][u + rt][t][kk], ii[t]);
          ri[t] = wy_mfma(A.a[0][f], w.x[1][u + rt][t][kk], ri[t]);
          ir[t] = wy_mfma(A.a[1][f], w.x[0][u + rt][t][kk], ir[t]);
        }
#pragma unroll
    for (int t = 0; t < T; ++t) {
      wr[t] = rr[t] - ii[t];
      wi[t] = ri[t] + ir[t];
    }
  }
  if (next) An.load(next);
  if constexpr (PL == 1) {
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int t = 0; t < T; ++t)
          w.x[0][u + rt][t] = wy_mfma(Vop.v[0][4 * rt + kk], wr[t][kk], w.x[0][u + rt][t]);
  } else {
    // X += V W':  re += Vr W're - Vi W'im,  im += Vr W'im + Vi W're
    V4 nwi[T];
#pragma unroll
    for (int t = 0; t < T; ++t) nwi[t] = -wi[t];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int t = 0; t < T; ++t) {
          const int f = 4 * rt + kk;
          w.x[0][u + rt][t] = wy_mfma(Vop.v[0][f], wr[t][kk], w.x[0][u + rt][t]);
          w.x[1][u + rt][t] = wy_mfma(Vop.v[0][f], wi[t][kk], w.x[1][u + rt][t]);
          w.x[0][u + rt][t] = wy_mfma(Vop.v[1][f], nwi[t][kk], w.x[0][u + rt][t]);
          w.x[1][u + rt][t] = wy_mfma(Vop.v[1][f], wr[t][kk], w.x[1][u + rt][t]);
        }
  }
}

// Chase steps [j0, j1) of block m on stripe c (j1 <= J0(m)); the stripe's
// row r is at Qs + (c rows_pad + r) SW.  The window's last row (row NB+K-1,
// which no reflector of the block touches) is read but never written: it may
// belong to another tile of the same launch.
template <typename E, int NB, int K, int T, bool PF, bool VP>
__device__ __forceinline__ void run_wy_steps(const typename WyElem<E>::R* __restrict__ P,
                                             const int64_t* __restrict__ Bt,
                                             E* __restrict__ Qs, int64_t rows_pad, int64_t c,
                                             int64_t m, int64_t j0, int64_t j1) {
  using Gm = WyGeom<NB, K>;
  using R = typename WyElem<E>::R;
  constexpr int SW = 16 * T, SG = Gm::SG, RTW = Gm::RTW, TN = NB / 16, TK = K / 16;
  constexpr int64_t REC = WyRec<E, NB, K>::REC;
  E* __restrict__ bp = Qs + c * rows_pad * SW;
  const int64_t s0 = m * K;
  const R* __restrict__ Pm = P + Bt[m] * (SG * REC);
  auto rec_of = [&](int64_t j, int u) -> const R* { return Pm + (j * SG + u) * REC; };
  WyWin<E, NB, K, T> w;
  // PF: the next step's NB new window rows are loaded at the start of a step
  // so that their memory latency overlaps the step's products (rows of this
  // tile's own range: no other tile of the launch touches them); without PF
  // (register budget) they load after the step
  typename WyElem<E>::V4 nx[WyElem<E>::PL][PF ? TN : 1][T];
  WyA<E, NB, K> A[2];
  WyV<E, NB, K> Vb[VP ? 2 : 1];
  A[0].load(rec_of(j0, SG - 1));
  if constexpr (VP) Vb[0].load(rec_of(j0, SG - 1));
  {
    const E* __restrict__ rp = bp + (s0 + 1 + j0 * NB) * SW;
#pragma unroll
    for (int tr = 0; tr < RTW; ++tr) wy_load_tile<E, NB, K, T, SW>(w, tr, rp);
  }
  for (int64_t j = j0; j < j1; ++j) {
    E* __restrict__ rp = bp + (s0 + 1 + j * NB) * SW;
    const R* next_step = (j + 1 < j1) ? rec_of(j + 1, SG - 1) : nullptr;
    if (PF && j + 1 < j1) {
      const E* __restrict__ np = rp + (NB + K) * SW;
      WyWin<E, NB, K, T> tmp;
#pragma unroll
      for (int tr = 0; tr < TN; ++tr) {
        wy_load_tile<E, NB, K, T, SW>(tmp, tr, np);
#pragma unroll
        for (int p = 0; p < WyElem<E>::PL; ++p)
#pragma unroll
          for (int t = 0; t < T; ++t) nx[p][tr][t] = tmp.x[p][tr][t];
      }
    }
    // sub-groups SG-1 .. 0; A[(SG-1-u) % 2] holds sub-group u's fragments
    RevFor<SG>::run([&](auto uc) {
      constexpr int u = decltype(uc)::value;
      constexpr int cur = (SG - 1 - u) & 1;
      const R* nx = (u > 0) ? rec_of(j, u - 1) : next_step;
      wy_subgroup<E, NB, K, T, u, VP>(w, A[cur], rec_of(j, u), nx, A[cur ^ 1], Vb[VP ? cur : 0],
                                      Vb[VP ? (cur ^ 1) : 0]);
    });
    // an odd sub-group count leaves the next step's first fragments in A[1]
    if constexpr ((SG & 1) == 1) {
      A[0] = A[1];
      if constexpr (VP) Vb[0] = Vb[1];
    }
    // rows final for this block
#pragma unroll
    for (int tr = 0; tr < TN; ++tr) wy_store_tile<E, NB, K, T, SW>(w, tr, rp, false);
    if (j + 1 < j1) {
      // carried tiles TN .. RTW-1 move to 0 .. TK-1; the next NB rows follow
#pragma unroll
      for (int p = 0; p < WyElem<E>::PL; ++p)
#pragma unroll
        for (int tr = 0; tr < TK; ++tr)
#pragma unroll
          for (int t = 0; t < T; ++t) w.x[p][tr][t] = w.x[p][tr + TN][t];
      if constexpr (PF) {
#pragma unroll
        for (int p = 0; p < WyElem<E>::PL; ++p)
#pragma unroll
          for (int tr = 0; tr < TN; ++tr)
#pragma unroll
            for (int t = 0; t < T; ++t) w.x[p][TK + tr][t] = nx[p][tr][t];
      } else {
        const E* __restrict__ np = rp + NB * SW;
#pragma unroll
        for (int tr = TK; tr < RTW; ++tr) wy_load_tile<E, NB, K, T, SW>(w, tr, np);
      }
    }
  }
  // carried rows (or final after the block's last step)
  E* __restrict__ rl = bp + (s0 + 1 + (j1 - 1) * NB) * SW;
#pragma unroll
  for (int tr = TN; tr < RTW; ++tr) wy_store_tile<E, NB, K, T, SW>(w, tr, rl, tr == RTW - 1);
}

template <typename E, int NB, int K, int T, int OCC, bool PF, bool VP>
__global__ __launch_bounds__(64, OCC) void k_wy(const typename WyElem<E>::R* __restrict__ P,
                                                const int64_t* __restrict__ Bt,
                                                E* __restrict__ Qs, int64_t rows_pad, int64_t n,
                                                int c0, int G, int M, int t, int m0, int S,
                                                int xcd) {
  const int b = tile_of((int)blockIdx.x, (int)gridDim.x, xcd);
  const int c = c0 + b % G;
  const int m = m0 + b / G;
  const int64_t J0 = block_steps(n, NB, K, m);
  const int64_t j0 = (int64_t)(t - (M - 1 - m)) * S;
  const int64_t j1 = (j0 + S < J0) ? j0 + S : J0;
  run_wy_steps<E, NB, K, T, PF, VP>(P, Bt, Qs, rows_pad, c, m, j0, j1);
}

template <typename E, int NB, int K, int T, int OCC, bool PF, bool VP>
__global__ __launch_bounds__(64, OCC) void k_wy_b(const ProblemDesc* __restrict__ d,
                                                  const DiagEntry* __restrict__ e, int ecount,
                                                  int t, int xcd) {
  const int b = tile_of((int)blockIdx.x, (int)gridDim.x, xcd);
  const DiagEntry& E0 = e[find_by<DiagEntry, &DiagEntry::tile0>(e, ecount, b)];
  const ProblemDesc& D = d[E0.p];
  const int local = b - E0.tile0;
  const int m = E0.m0 + local / D.G;
  const int64_t J0 = block_steps(D.n, NB, K, m);
  const int64_t j0 = (int64_t)(t - (D.M - 1 - m)) * D.S;
  const int64_t j1 = (j0 + D.S < J0) ? j0 + D.S : J0;
  run_wy_steps<E, NB, K, T, PF, VP>((const typename WyElem<E>::R*)D.P, (const int64_t*)D.Bt, (E*)D.Qs,
                            D.rows_pad, local % D.G, m, j0, j1);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// Packed area of one problem: the records of every block's existing steps
// back to back, then the block table Bt[0..M).
template <typename E, int NB, int K>
size_t wy_rbytes(int64_t n) {
  const int64_t M = (n - 1 + K - 1) / K;
  return align256((size_t)block_base(n, NB, K, M) * WyGeom<NB, K>::SG *
                  WyRec<E, NB, K>::REC * sizeof(typename WyElem<E>::R));
}

template <typename E, int NB, int K>
size_t wy_pbytes(int64_t n) {
  const int64_t M = (n - 1 + K - 1) / K;
  return wy_rbytes<E, NB, K>(n) + align256((size_t)M * sizeof(int64_t));
}

template <typename E, int NB, int K, int T>
size_t wy_workspace(int64_t n, int64_t nev) {
  const DiagPlan pl(n, nev, NB, K, 1, 16 * T);
  return wy_pbytes<E, NB, K>(n) + pl.template qbytes<E>();
}

// Single problem.  ws_in: a device workspace of at least
// wy_workspace(n, nev) bytes that no other work uses while this call's work
// runs, or null: then the workspace is allocated and freed in stream order.
template <typename E, int NB, int K, int T, int OCC, bool PF, bool VP>
hipError_t run_wy(const void* hh, const void* tau, void* Q, int64_t ldq, int64_t n,
                  int64_t nev, TileOpts opt, hipStream_t st, int num_cu, void* ws_in) {
  using Gm = WyGeom<NB, K>;
  using R = typename WyElem<E>::R;
  constexpr int SW = 16 * T;
  static const int64_t slots = wave_slots(k_wy<E, NB, K, T, OCC, PF, VP>, num_cu);
  const int64_t S = opt.steps > 0 ? opt.steps : choose_steps(n, nev, NB, K, slots, SW);
  const DiagPlan pl(n, nev, NB, K, S, SW);
  const int64_t Jmax = (n - 1 + NB - 1) / NB;
  if (pl.G * pl.M >= INT32_MAX || pl.M * Jmax * Gm::SG >= INT32_MAX || n + NB + K >= INT32_MAX)
    return hipErrorInvalidValue;
  const size_t rbytes = wy_rbytes<E, NB, K>(n), pbytes = wy_pbytes<E, NB, K>(n);
  char* ws = (char*)ws_in;
  hipError_t err = hipSuccess;
  if (!ws_in) {
    err = ws_alloc((void**)&ws, pbytes + pl.template qbytes<E>(), st);
    if (err != hipSuccess) return err;
  }
  auto release = [&](hipError_t e) {
    if (!ws_in) {
      const hipError_t e2 = ws_free(ws, st);
      if (e == hipSuccess) e = e2;
    }
    return e;
  };
  R* Pk = (R*)ws;
  int64_t* Bt = (int64_t*)(ws + rbytes);
  E* Qs = (E*)(ws + pbytes);
  const unsigned gt = (unsigned)((nev + 63) / 64);
  hipLaunchKernelGGL((k_wy_prep<E, NB, K>), dim3((unsigned)(pl.M * Jmax * Gm::SG)), dim3(256), 0,
                     st, (const E*)hh, (const E*)tau, n, Jmax, Pk, Bt);
  hipLaunchKernelGGL((k_to_rows_sw<E, SW>), dim3((unsigned)(pl.rows_pad / 64), gt), dim3(256), 0,
                     st, (const E*)Q, ldq, n, nev, Qs, pl.rows_pad, pl.G);
  const int ns = (int)std::max<int64_t>(1, std::min<int64_t>(opt.streams, pl.G));
  ProfScope prof(st, K, S, ns);
  {
    StreamFork fork(st, ns);
    if (fork.error() != hipSuccess) return release(fork.error());
    for (int64_t t = 0; t < pl.T; ++t) {
      int64_t m0, cnt;
      pl.active(t, &m0, &cnt);
      if (cnt == 0) continue;
      for (int i = 0; i < ns; ++i) {
        const int64_t c_lo = pl.G * i / ns, gs = pl.G * (i + 1) / ns - c_lo;
        prof.before(fork.stream(i));
        hipLaunchKernelGGL((k_wy<E, NB, K, T, OCC, PF, VP>), dim3((unsigned)(cnt * gs)), dim3(64), 0,
                           fork.stream(i), (const R*)Pk, (const int64_t*)Bt, Qs, pl.rows_pad, n,
                           (int)c_lo, (int)gs, (int)pl.M, (int)t, (int)m0, (int)S, opt.xcd);
        prof.after(fork.stream(i));
      }
    }
    err = fork.join();
  }
  prof.end();
  if (err != hipSuccess) return release(err);
  hipLaunchKernelGGL((k_from_rows_sw<E, SW>), dim3((unsigned)((n + 63) / 64), gt), dim3(256), 0,
                     st, (const E*)Qs, pl.rows_pad, (E*)Q, ldq, n, nev, pl.G);
  return release(hipGetLastError());
}

template <typename E, int NB, int K, int T, int OCC, bool PF, bool VP>
hipError_t launch_wy(const void* hh, const void* tau, void* Q, int64_t ldq, int64_t n,
                     int64_t nev, TileOpts opt, hipStream_t st, int num_cu) {
  return run_wy<E, NB, K, T, OCC, PF, VP>(hh, tau, Q, ldq, n, nev, opt, st, num_cu, nullptr);
}

template <typename E, int NB, int K, int T, int OCC, bool PF, bool VP>
hipError_t launch_wy_ws(const void* hh, const void* tau, void* Q, int64_t ldq, int64_t n,
                        int64_t nev, TileOpts opt, hipStream_t st, int num_cu, void* ws) {
  return run_wy<E, NB, K, T, OCC, PF, VP>(hh, tau, Q, ldq, n, nev, opt, st, num_cu, ws);
}

// Batched: problems idx[0..cnt) of probs (element type E, semi-bandwidth NB,
// validated by the caller); all problems' diagonal schedules side by side.
template <typename E, int NB, int K, int T, int OCC, bool PF, bool VP>
hipError_t launch_wy_batched(const elpa_hh_problem* probs, const int64_t* idx, int64_t cnt,
                             TileOpts opt, hipStream_t st, int num_cu) {
  using Gm = WyGeom<NB, K>;
  constexpr int SW = 16 * T;
  const int64_t S = opt.steps;
  static const int64_t slots = wave_slots(k_wy_b<E, NB, K, T, OCC, PF, VP>, num_cu);
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
    const int64_t s = S > 0 ? S : choose_steps(p.n, total_cols, NB, K, slots, SW);
    plans.emplace_back(p.n, p.nev, NB, K, s, SW);
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
  int64_t T_ = 0;
  std::vector<size_t> pat(d.size()), qat(d.size()), rb(d.size());
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
    rb[i] = wy_rbytes<E, NB, K>(pl.n);
    off += wy_pbytes<E, NB, K>(pl.n);
    qat[i] = off;
    off += pl.template qbytes<E>();
    T_ = std::max(T_, pl.T);
  }
  std::vector<DiagEntry> ent;
  std::vector<int64_t> eoff((size_t)T_ + 1, 0), etiles((size_t)T_, 0);
  for (int64_t t = 0; t < T_; ++t) {
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
  eoff[(size_t)T_] = (int64_t)ent.size();
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
    d[i].Bt = ws + dbytes + ebytes + pat[i] + rb[i];
    d[i].Qs = ws + dbytes + ebytes + qat[i];
  }
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
  hipLaunchKernelGGL((k_wy_prep_b<E, NB, K>), dim3((unsigned)ptiles), dim3(256), 0, st, dd, count);
  hipLaunchKernelGGL((k_to_rows_sw_b<E, SW>), dim3((unsigned)tiles), dim3(256), 0, st, dd, count);
  {
    ProfScope prof(st, K, S);
    for (int64_t t = 0; t < T_; ++t) {
      const int64_t ne = eoff[(size_t)t + 1] - eoff[(size_t)t];
      if (ne == 0) continue;
      prof.before(st);
      hipLaunchKernelGGL((k_wy_b<E, NB, K, T, OCC, PF, VP>), dim3((unsigned)etiles[(size_t)t]), dim3(64), 0,
                         st, dd, de + eoff[(size_t)t], (int)ne, (int)t, opt.xcd);
      prof.after(st);
    }
  }
  hipLaunchKernelGGL((k_from_rows_sw_b<E, SW>), dim3((unsigned)otiles), dim3(256), 0, st, dd,
                     count);
  err = hipGetLastError();
  const hipError_t e2 = ws_free(ws, st);
  return err != hipSuccess ? err : e2;
}

}  // namespace ehh
