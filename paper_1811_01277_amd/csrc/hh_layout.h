// Layout conversion between the caller's Q (column major) and the stripe-major
// workspace of the stripe kernels: stripe c holds columns [SW c, SW c + SW) as
// a contiguous rows_pad x SW row-major block, so a row of a stripe is one
// contiguous access and window rows sit at a constant stride.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hh_sched.h"

namespace ehh {

// Layout conversion between Q (column major) and SW-column stripes, element
// (r, SW*c + l) at Qs[(c*rows_pad + r)*SW + l]; 64 x 64 tiles through LDS,
// padding rows and columns written as zeros.
template <typename E, int SW>
__device__ __forceinline__ void to_rows_tile_sw(const E* __restrict__ Q, int64_t ldq,
                                                int64_t n, int64_t nev, E* __restrict__ Qs,
                                                int64_t rows_pad, int64_t G, int64_t rt,
                                                int64_t ct, E (*tile)[65]) {
  const int64_t r0 = rt * 64, c0 = ct * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int cc = ty; cc < 64; cc += 4) {
    const int64_t r = r0 + tx, col = c0 + cc;
    tile[cc][tx] = (r < n && col < nev) ? Q[r + col * ldq] : E{};
  }
  __syncthreads();
  const int64_t col = c0 + tx, c = col / SW, l = col - c * SW;
  if (c >= G) return;
  E* __restrict__ dst = Qs + c * rows_pad * SW + l;
  for (int rr = ty; rr < 64; rr += 4) {
    const int64_t r = r0 + rr;
    if (r < rows_pad) dst[r * SW] = tile[tx][rr];
  }
}

template <typename E, int SW>
__device__ __forceinline__ void from_rows_tile_sw(const E* __restrict__ Qs, int64_t rows_pad,
                                                  E* __restrict__ Q, int64_t ldq, int64_t n,
                                                  int64_t nev, int64_t G, int64_t rt, int64_t ct,
                                                  E (*tile)[65]) {
  const int64_t r0 = rt * 64, c0 = ct * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  {
    const int64_t col = c0 + tx, c = col / SW, l = col - c * SW;
    for (int rr = ty; rr < 64; rr += 4) {
      const int64_t r = r0 + rr;
      if (r < n && c < G) tile[rr][tx] = Qs[(c * rows_pad + r) * SW + l];
    }
  }
  __syncthreads();
  for (int cc = ty; cc < 64; cc += 4) {
    const int64_t r = r0 + tx, col = c0 + cc;
    if (r < n && col < nev) Q[r + col * ldq] = tile[tx][cc];
  }
}

template <typename E, int SW>
__global__ __launch_bounds__(256) void k_to_rows_sw(const E* __restrict__ Q, int64_t ldq,
                                                    int64_t n, int64_t nev,
                                                    E* __restrict__ Qs, int64_t rows_pad,
                                                    int64_t G) {
  __shared__ E tile[64][65];
  to_rows_tile_sw<E, SW>(Q, ldq, n, nev, Qs, rows_pad, G, blockIdx.x, blockIdx.y, tile);
}

template <typename E, int SW>
__global__ __launch_bounds__(256) void k_from_rows_sw(const E* __restrict__ Qs,
                                                      int64_t rows_pad, E* __restrict__ Q,
                                                      int64_t ldq, int64_t n, int64_t nev,
                                                      int64_t G) {
  __shared__ E tile[64][65];
  from_rows_tile_sw<E, SW>(Qs, rows_pad, Q, ldq, n, nev, G, blockIdx.x, blockIdx.y, tile);
}

template <typename E, int SW>
__global__ __launch_bounds__(256) void k_to_rows_sw_b(const ProblemDesc* __restrict__ d,
                                                      int count) {
  __shared__ E tile[64][65];
  const int t = (int)blockIdx.x;
  const ProblemDesc& D = d[find_by<ProblemDesc, &ProblemDesc::tile0>(d, count, t)];
  const int local = t - D.tile0;
  to_rows_tile_sw<E, SW>((const E*)D.Q, D.ldq, D.n, D.nev, (E*)D.Qs, D.rows_pad, D.G,
                      local / D.GT, local % D.GT, tile);
}

template <typename E, int SW>
__global__ __launch_bounds__(256) void k_from_rows_sw_b(const ProblemDesc* __restrict__ d,
                                                        int count) {
  __shared__ E tile[64][65];
  const int t = (int)blockIdx.x;
  const ProblemDesc& D = d[find_by<ProblemDesc, &ProblemDesc::otile0>(d, count, t)];
  const int local = t - D.otile0;
  from_rows_tile_sw<E, SW>((const E*)D.Qs, D.rows_pad, (E*)D.Q, D.ldq, D.n, D.nev, D.G,
                        local / D.GT, local % D.GT, tile);
}

}  // namespace ehh
