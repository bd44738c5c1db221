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
