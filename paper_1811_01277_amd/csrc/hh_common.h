// Shared device/host helpers of the tridiagonal->band back-transformation
// kernels: slot arithmetic of the bulge-chase reflectors and the element
// operations for real (float, double) and complex double values.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ehh {

// C(M) = sum_{m=1..M} ceil(m / b).  With J(s) = ceil((n-1-s)/b) chase steps in
// sweep s, the first slot of sweep s is sum_{s'<s} J(s') = C(n-1) - C(n-1-s),
// and the number of slots is C(n-1).
__host__ __device__ __forceinline__ int64_t csum(int64_t M, int64_t b) {
  const int64_t q = M / b, r = M - q * b;
  return b * q * (q + 1) / 2 + r * (q + 1);
}

__host__ __device__ __forceinline__ int64_t slot_offset(int64_t n, int64_t b, int64_t s) {
  return csum(n - 1, b) - csum(n - 1 - s, b);
}

// F(N, d, a, c) = sum_{i=0}^{N-1} floor((a i + c) / d) for a, c >= 0, d > 0,
// by the Euclid-like reduction of lattice-point counts: whole multiples of d
// in a and c contribute in closed form; with a, c < d the count of points
// under the line y = (a x + c)/d, x < N, equals the count under the
// transposed line with the roles of a and d exchanged, over
// floor((a N + c)/d) columns.  O(log d) iterations.
__host__ __device__ __forceinline__ int64_t floor_sum(int64_t N, int64_t d, int64_t a,
                                                     int64_t c) {
  int64_t s = 0;
  while (N > 0) {
    if (a >= d) {
      s += (a / d) * (N * (N - 1) / 2);
      a %= d;
    }
    if (c >= d) {
      s += (c / d) * N;
      c %= d;
    }
    const int64_t top = a * N + c;
    if (top < d) break;
    N = top / d;
    c = top % d;
    const int64_t t = d;
    d = a;
    a = t;
  }
  return s;
}

// Chase steps of sweep block m (sweeps [mK, mK+K)): J0(m) = ceil((n-1-mK)/b),
// the steps of its first (longest) sweep.
__host__ __device__ __forceinline__ int64_t block_steps(int64_t n, int64_t b, int64_t K,
                                                       int64_t m) {
  return (n - 1 - m * K + b - 1) / b;
}

// sum_{m' < m} J0(m'): the first packed step record of block m when the
// records of every block's existing steps are stored back to back (0 <= m <=
// M = ceil((n-1)/K); m = M gives the total).  With i = m-1-m' the terms are
// floor((K i + n-2+b-(m-1)K) / b), whose offset is >= b-1 for m <= M.
__host__ __device__ __forceinline__ int64_t block_base(int64_t n, int64_t b, int64_t K,
                                                      int64_t m) {
  if (m <= 0) return 0;
  return floor_sum(m, b, K, n - 2 + b - (m - 1) * K);
}

struct z64 {
  double re, im;
};

// Element operations.  dot: acc += conj(v) * x;  scale: tau * w;
// axpy: x -= v * w.  The reflector value v is wave-uniform.
template <typename E>
struct Ops;

template <>
struct Ops<double> {
  using E = double;
  static __device__ __forceinline__ E zero() { return 0.0; }
  static __device__ __forceinline__ void dot(E& acc, E v, E x) { acc = __builtin_fma(v, x, acc); }
  static __device__ __forceinline__ E add(E a, E b) { return a + b; }
  static __device__ __forceinline__ E scale(E w, E t) { return w * t; }
  static __device__ __forceinline__ void axpy(E& x, E v, E w) { x = __builtin_fma(-v, w, x); }
};

template <>
struct Ops<float> {
  using E = float;
  static __device__ __forceinline__ E zero() { return 0.0f; }
  static __device__ __forceinline__ void dot(E& acc, E v, E x) { acc = __builtin_fmaf(v, x, acc); }
  static __device__ __forceinline__ E add(E a, E b) { return a + b; }
  static __device__ __forceinline__ E scale(E w, E t) { return w * t; }
  static __device__ __forceinline__ void axpy(E& x, E v, E w) { x = __builtin_fmaf(-v, w, x); }
};

template <>
struct Ops<z64> {
  using E = z64;
  static __device__ __forceinline__ E zero() { return E{0.0, 0.0}; }
  static __device__ __forceinline__ void dot(E& acc, E v, E x) {
    // conj(v) * x = (vr xr + vi xi) + i (vr xi - vi xr)
    acc.re = __builtin_fma(v.re, x.re, acc.re);
    acc.re = __builtin_fma(v.im, x.im, acc.re);
    acc.im = __builtin_fma(v.re, x.im, acc.im);
    acc.im = __builtin_fma(-v.im, x.re, acc.im);
  }
  static __device__ __forceinline__ E add(E a, E b) { return E{a.re + b.re, a.im + b.im}; }
  static __device__ __forceinline__ E scale(E w, E t) {
    return E{t.re * w.re - t.im * w.im, t.re * w.im + t.im * w.re};
  }
  static __device__ __forceinline__ void axpy(E& x, E v, E w) {
    // x -= v * w = (vr wr - vi wi) + i (vr wi + vi wr)
    x.re = __builtin_fma(-v.re, w.re, x.re);
    x.re = __builtin_fma(v.im, w.im, x.re);
    x.im = __builtin_fma(-v.re, w.im, x.im);
    x.im = __builtin_fma(-v.im, w.re, x.im);
  }
};

}  // namespace ehh
