// fp64 FMA blocks whose reflector operand is broadcast from a VGPR with the
// DPP row_newbcast modifier (gfx90a and later; 64-bit DPP supports this one
// control).  A reflector segment of 16 values is held in one 64-bit VGPR
// pair, replicated in the four 16-lane rows of the wave: lane 16r+i holds
// v[i].  row_newbcast:i hands lane i of each row to the whole row, so every
// lane sees v[i] as the first FMA operand without a scalar load.  The values
// arrive through ordinary vector loads, whose in-order completion lets a
// reflector be prefetched a full reflector ahead (scalar loads can return
// out of order, so every wait on them is a wait for all of them).
//
// Each block starts with s_nop 1: two wait states between a VALU write of a
// DPP source register and the DPP read.
#pragma once

#include <hip/hip_runtime.h>

#include "hh_common.h"

namespace ehh {

// the broadcast lane is an immediate asm operand (operand number N)
#define EHH_DPP(N) " row_newbcast:%" #N " row_mask:0xf bank_mask:0xf\n"

// a_g += bcast(V_g, I) * x_g for g = 0..3 (x_g: window element of v index 16g+I).
template <int I>
__device__ __forceinline__ void dpp_dot4(double& a0, double& a1, double& a2, double& a3, double V0,
                                         double V1, double V2, double V3, const double* x0,
                                         const double* x1, const double* x2, const double* x3) {
  asm volatile("s_nop 1\n"
               "v_fmac_f64_dpp %0, %4, %8" EHH_DPP(12)
               "v_fmac_f64_dpp %1, %5, %9" EHH_DPP(12)
               "v_fmac_f64_dpp %2, %6, %10" EHH_DPP(12)
               "v_fmac_f64_dpp %3, %7, %11" EHH_DPP(12)
               : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3)
               : "v"(V0), "v"(V1), "v"(V2), "v"(V3), "v"(x0[0]), "v"(x1[0]), "v"(x2[0]),
                 "v"(x3[0]), "i"(I));
}

// x_g += bcast(V_g, I) * nw for g = 0..3 (nw = -tau * dot).
template <int I>
__device__ __forceinline__ void dpp_upd4(double& x0, double& x1, double& x2, double& x3, double V0,
                                         double V1, double V2, double V3, double nw) {
  asm volatile("s_nop 1\n"
               "v_fmac_f64_dpp %0, %4, %8" EHH_DPP(9)
               "v_fmac_f64_dpp %1, %5, %8" EHH_DPP(9)
               "v_fmac_f64_dpp %2, %6, %8" EHH_DPP(9)
               "v_fmac_f64_dpp %3, %7, %8" EHH_DPP(9)
               : "+v"(x0), "+v"(x1), "+v"(x2), "+v"(x3)
               : "v"(V0), "v"(V1), "v"(V2), "v"(V3), "v"(nw), "i"(I));
}

// two-segment variants (NB = 32)
template <int I>
__device__ __forceinline__ void dpp_dot2(double& a0, double& a1, double V0, double V1,
                                         const double* x0, const double* x1) {
  asm volatile("s_nop 1\n"
               "v_fmac_f64_dpp %0, %2, %4" EHH_DPP(6)
               "v_fmac_f64_dpp %1, %3, %5" EHH_DPP(6)
               : "+v"(a0), "+v"(a1)
               : "v"(V0), "v"(V1), "v"(x0[0]), "v"(x1[0]), "i"(I));
}

template <int I>
__device__ __forceinline__ void dpp_upd2(double& x0, double& x1, double V0, double V1, double nw) {
  asm volatile("s_nop 1\n"
               "v_fmac_f64_dpp %0, %2, %4" EHH_DPP(5)
               "v_fmac_f64_dpp %1, %3, %4" EHH_DPP(5)
               : "+v"(x0), "+v"(x1)
               : "v"(V0), "v"(V1), "v"(nw), "i"(I));
}

// ---------------------------------------------------------------------------
// Split-window blocks (two lanes per column, rows interleaved by parity).
// A reflector's values for one lane half arrive as 16-value segments held in
// VGPR pairs (lane 16r+i holds segment value i); each block below covers
// broadcast lanes l0..l7 of one or two segments, so a reflector takes two
// blocks per pass and one s_nop per 8 or 16 FMAs.  The _X forms add the
// extra term of an odd window offset: segment 2's lane-0 value against one
// more window row.
// ---------------------------------------------------------------------------
#define EHH_F(D, S, X, L) \
  "v_fmac_f64_dpp %" #D ", %" #S ", %" #X " row_newbcast:" #L " row_mask:0xf bank_mask:0xf\n"
#define EHH_X(m, ...) m(__VA_ARGS__)
#define EHH_LA 0, 1, 2, 3, 4, 5, 6, 7
#define EHH_LB 8, 9, 10, 11, 12, 13, 14, 15
#define EHH_VX8(p) \
  "v"(p[0]), "v"(p[1]), "v"(p[2]), "v"(p[3]), "v"(p[4]), "v"(p[5]), "v"(p[6]), "v"(p[7])
#define EHH_PX8(p)                                                                        \
  "+v"(p[0]), "+v"(p[1]), "+v"(p[2]), "+v"(p[3]), "+v"(p[4]), "+v"(p[5]), "+v"(p[6]), \
      "+v"(p[7])

// one segment: a0/a1 += bcast(V0, l) * x  (%0 a0, %1 a1, %2 V0, %3..%10 x)
#define EHH_SDOT1(l0, l1, l2, l3, l4, l5, l6, l7)                                      \
  EHH_F(0, 2, 3, l0) EHH_F(1, 2, 4, l1) EHH_F(0, 2, 5, l2) EHH_F(1, 2, 6, l3)          \
  EHH_F(0, 2, 7, l4) EHH_F(1, 2, 8, l5) EHH_F(0, 2, 9, l6) EHH_F(1, 2, 10, l7)
// one segment: x += bcast(V, l) * nw  (%0..%7 x)
#define EHH_SUPD1(V, NW, l0, l1, l2, l3, l4, l5, l6, l7)                                \
  EHH_F(0, V, NW, l0) EHH_F(1, V, NW, l1) EHH_F(2, V, NW, l2) EHH_F(3, V, NW, l3)      \
  EHH_F(4, V, NW, l4) EHH_F(5, V, NW, l5) EHH_F(6, V, NW, l6) EHH_F(7, V, NW, l7)
// two segments: a0 += bcast(V0, l) * x, a1 += bcast(V1, l) * y
// (%0 a0, %1 a1, %2 V0, %3 V1, %4..%11 x, %12..%19 y)
#define EHH_SDOT2(l0, l1, l2, l3, l4, l5, l6, l7)                                      \
  EHH_F(0, 2, 4, l0) EHH_F(1, 3, 12, l0) EHH_F(0, 2, 5, l1) EHH_F(1, 3, 13, l1)        \
  EHH_F(0, 2, 6, l2) EHH_F(1, 3, 14, l2) EHH_F(0, 2, 7, l3) EHH_F(1, 3, 15, l3)        \
  EHH_F(0, 2, 8, l4) EHH_F(1, 3, 16, l4) EHH_F(0, 2, 9, l5) EHH_F(1, 3, 17, l5)        \
  EHH_F(0, 2, 10, l6) EHH_F(1, 3, 18, l6) EHH_F(0, 2, 11, l7) EHH_F(1, 3, 19, l7)
// two segments: x += bcast(V0, l) * nw, y += bcast(V1, l) * nw (%0..%7 x, %8..%15 y)
#define EHH_SUPD2(V0, V1, NW, l0, l1, l2, l3, l4, l5, l6, l7)                                 \
  EHH_F(0, V0, NW, l0) EHH_F(8, V1, NW, l0) EHH_F(1, V0, NW, l1) EHH_F(9, V1, NW, l1)        \
  EHH_F(2, V0, NW, l2) EHH_F(10, V1, NW, l2) EHH_F(3, V0, NW, l3) EHH_F(11, V1, NW, l3)      \
  EHH_F(4, V0, NW, l4) EHH_F(12, V1, NW, l4) EHH_F(5, V0, NW, l5) EHH_F(13, V1, NW, l5)      \
  EHH_F(6, V0, NW, l6) EHH_F(14, V1, NW, l6) EHH_F(7, V0, NW, l7) EHH_F(15, V1, NW, l7)

// dot, one segment, lanes 0..7 and lanes 8..15 (+ extra term when EX)
__device__ __forceinline__ void sdot1_a(double& a0, double& a1, double V0, const double* x) {
  asm volatile("s_nop 1\n" EHH_X(EHH_SDOT1, EHH_LA) : "+v"(a0), "+v"(a1) : "v"(V0), EHH_VX8(x));
}
template <bool EX>
__device__ __forceinline__ void sdot1_b(double& a0, double& a1, double V0, double V2,
                                        const double* x, const double* xe) {
  if constexpr (EX)
    asm volatile("s_nop 1\n" EHH_X(EHH_SDOT1, EHH_LB) EHH_F(0, 11, 12, 0)
                 : "+v"(a0), "+v"(a1)
                 : "v"(V0), EHH_VX8(x), "v"(V2), "v"(xe[0]));
  else
    asm volatile("s_nop 1\n" EHH_X(EHH_SDOT1, EHH_LB) : "+v"(a0), "+v"(a1) : "v"(V0), EHH_VX8(x));
}
// update, one segment
__device__ __forceinline__ void supd1_a(double* x, double V0, double nw) {
  asm volatile("s_nop 1\n" EHH_X(EHH_SUPD1, 8, 9, EHH_LA) : EHH_PX8(x) : "v"(V0), "v"(nw));
}
template <bool EX>
__device__ __forceinline__ void supd1_b(double* x, double* xe, double V0, double V2, double nw) {
  if constexpr (EX)
    asm volatile("s_nop 1\n" EHH_X(EHH_SUPD1, 9, 10, EHH_LB) EHH_F(8, 11, 10, 0)
                 : EHH_PX8(x), "+v"(xe[0])
                 : "v"(V0), "v"(nw), "v"(V2));
  else
    asm volatile("s_nop 1\n" EHH_X(EHH_SUPD1, 8, 9, EHH_LB) : EHH_PX8(x) : "v"(V0), "v"(nw));
}
// dot, two segments
__device__ __forceinline__ void sdot2_a(double& a0, double& a1, double V0, double V1,
                                        const double* x, const double* y) {
  asm volatile("s_nop 1\n" EHH_X(EHH_SDOT2, EHH_LA)
               : "+v"(a0), "+v"(a1)
               : "v"(V0), "v"(V1), EHH_VX8(x), EHH_VX8(y));
}
template <bool EX>
__device__ __forceinline__ void sdot2_b(double& a0, double& a1, double V0, double V1, double V2,
                                        const double* x, const double* y, const double* xe) {
  if constexpr (EX)
    asm volatile("s_nop 1\n" EHH_X(EHH_SDOT2, EHH_LB) EHH_F(0, 20, 21, 0)
                 : "+v"(a0), "+v"(a1)
                 : "v"(V0), "v"(V1), EHH_VX8(x), EHH_VX8(y), "v"(V2), "v"(xe[0]));
  else
    asm volatile("s_nop 1\n" EHH_X(EHH_SDOT2, EHH_LB)
                 : "+v"(a0), "+v"(a1)
                 : "v"(V0), "v"(V1), EHH_VX8(x), EHH_VX8(y));
}
// update, two segments
__device__ __forceinline__ void supd2_a(double* x, double* y, double V0, double V1, double nw) {
  asm volatile("s_nop 1\n" EHH_X(EHH_SUPD2, 16, 17, 18, EHH_LA)
               : EHH_PX8(x), EHH_PX8(y)
               : "v"(V0), "v"(V1), "v"(nw));
}
template <bool EX>
__device__ __forceinline__ void supd2_b(double* x, double* y, double* xe, double V0, double V1,
                                        double V2, double nw) {
  if constexpr (EX)
    asm volatile("s_nop 1\n" EHH_X(EHH_SUPD2, 17, 18, 19, EHH_LB) EHH_F(16, 20, 19, 0)
                 : EHH_PX8(x), EHH_PX8(y), "+v"(xe[0])
                 : "v"(V0), "v"(V1), "v"(nw), "v"(V2));
  else
    asm volatile("s_nop 1\n" EHH_X(EHH_SUPD2, 16, 17, 18, EHH_LB)
                 : EHH_PX8(x), EHH_PX8(y)
                 : "v"(V0), "v"(V1), "v"(nw));
}

// ---------------------------------------------------------------------------
// Complex (fp64 pairs) split-window blocks.  One segment, broadcast lanes
// l0..l0+7: dot  a += conj(v) x  (4 FMAs per value, the -Im v term through the
// DPP source's negation modifier); update  x += v nw  (nw = -tau a, 4 FMAs).
// Operands: dot %0 a.re, %1 a.im, %2 V.re, %3 V.im, %4.. x[k].re, x[k].im;
// update %0.. x[k].re, x[k].im, then V.re, V.im, nw.re, nw.im.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void cdot_a(double& ar, double& ai, double Vr, double Vi,
                                       const z64* x) {
  asm volatile("s_nop 1\n"
               "v_fmac_f64_dpp %0, %2, %4 row_newbcast:0 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, %2, %5 row_newbcast:0 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %0, %3, %5 row_newbcast:0 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, -%3, %4 row_newbcast:0 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %0, %2, %6 row_newbcast:1 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, %2, %7 row_newbcast:1 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %0, %3, %7 row_newbcast:1 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, -%3, %6 row_newbcast:1 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %0, %2, %8 row_newbcast:2 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, %2, %9 row_newbcast:2 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %0, %3, %9 row_newbcast:2 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, -%3, %8 row_newbcast:2 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %0, %2, %10 row_newbcast:3 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, %2, %11 row_newbcast:3 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %0, %3, %11 row_newbcast:3 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, -%3, %10 row_newbcast:3 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %0, %2, %12 row_newbcast:4 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, %2, %13 row_newbcast:4 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %0, %3, %13 row_newbcast:4 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, -%3, %12 row_newbcast:4 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %0, %2, %14 row_newbcast:5 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, %2, %15 row_newbcast:5 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %0, %3, %15 row_newbcast:5 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, -%3, %14 row_newbcast:5 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %0, %2, %16 row_newbcast:6 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, %2, %17 row_newbcast:6 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %0, %3, %17 row_newbcast:6 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, -%3, %16 row_newbcast:6 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %0, %2, %18 row_newbcast:7 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, %2, %19 row_newbcast:7 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %0, %3, %19 row_newbcast:7 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, -%3, %18 row_newbcast:7 row_mask:0xf bank_mask:0xf\n"
               : "+v"(ar), "+v"(ai)
               : "v"(Vr), "v"(Vi), "v"(x[0].re), "v"(x[0].im), "v"(x[1].re), "v"(x[1].im), "v"(x[2].re), "v"(x[2].im), "v"(x[3].re), "v"(x[3].im), "v"(x[4].re), "v"(x[4].im), "v"(x[5].re), "v"(x[5].im), "v"(x[6].re), "v"(x[6].im), "v"(x[7].re), "v"(x[7].im));
}
__device__ __forceinline__ void cupd_a(z64* x, double Vr, double Vi, double nr,
                                       double ni) {
  asm volatile("s_nop 1\n"
               "v_fmac_f64_dpp %0, %16, %18 row_newbcast:0 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, %16, %19 row_newbcast:0 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %0, -%17, %19 row_newbcast:0 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, %17, %18 row_newbcast:0 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %2, %16, %18 row_newbcast:1 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %3, %16, %19 row_newbcast:1 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %2, -%17, %19 row_newbcast:1 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %3, %17, %18 row_newbcast:1 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %4, %16, %18 row_newbcast:2 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %5, %16, %19 row_newbcast:2 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %4, -%17, %19 row_newbcast:2 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %5, %17, %18 row_newbcast:2 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %6, %16, %18 row_newbcast:3 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %7, %16, %19 row_newbcast:3 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %6, -%17, %19 row_newbcast:3 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %7, %17, %18 row_newbcast:3 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %8, %16, %18 row_newbcast:4 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %9, %16, %19 row_newbcast:4 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %8, -%17, %19 row_newbcast:4 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %9, %17, %18 row_newbcast:4 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %10, %16, %18 row_newbcast:5 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %11, %16, %19 row_newbcast:5 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %10, -%17, %19 row_newbcast:5 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %11, %17, %18 row_newbcast:5 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %12, %16, %18 row_newbcast:6 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %13, %16, %19 row_newbcast:6 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %12, -%17, %19 row_newbcast:6 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %13, %17, %18 row_newbcast:6 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %14, %16, %18 row_newbcast:7 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %15, %16, %19 row_newbcast:7 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %14, -%17, %19 row_newbcast:7 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %15, %17, %18 row_newbcast:7 row_mask:0xf bank_mask:0xf\n"
               : "+v"(x[0].re), "+v"(x[0].im), "+v"(x[1].re), "+v"(x[1].im), "+v"(x[2].re), "+v"(x[2].im), "+v"(x[3].re), "+v"(x[3].im), "+v"(x[4].re), "+v"(x[4].im), "+v"(x[5].re), "+v"(x[5].im), "+v"(x[6].re), "+v"(x[6].im), "+v"(x[7].re), "+v"(x[7].im)
               : "v"(Vr), "v"(Vi), "v"(nr), "v"(ni));
}
__device__ __forceinline__ void cdot_b(double& ar, double& ai, double Vr, double Vi,
                                       const z64* x) {
  asm volatile("s_nop 1\n"
               "v_fmac_f64_dpp %0, %2, %4 row_newbcast:8 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, %2, %5 row_newbcast:8 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %0, %3, %5 row_newbcast:8 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, -%3, %4 row_newbcast:8 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %0, %2, %6 row_newbcast:9 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, %2, %7 row_newbcast:9 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %0, %3, %7 row_newbcast:9 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, -%3, %6 row_newbcast:9 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %0, %2, %8 row_newbcast:10 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, %2, %9 row_newbcast:10 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %0, %3, %9 row_newbcast:10 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, -%3, %8 row_newbcast:10 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %0, %2, %10 row_newbcast:11 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, %2, %11 row_newbcast:11 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %0, %3, %11 row_newbcast:11 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, -%3, %10 row_newbcast:11 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %0, %2, %12 row_newbcast:12 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, %2, %13 row_newbcast:12 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %0, %3, %13 row_newbcast:12 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, -%3, %12 row_newbcast:12 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %0, %2, %14 row_newbcast:13 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, %2, %15 row_newbcast:13 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %0, %3, %15 row_newbcast:13 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, -%3, %14 row_newbcast:13 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %0, %2, %16 row_newbcast:14 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, %2, %17 row_newbcast:14 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %0, %3, %17 row_newbcast:14 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, -%3, %16 row_newbcast:14 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %0, %2, %18 row_newbcast:15 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, %2, %19 row_newbcast:15 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %0, %3, %19 row_newbcast:15 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, -%3, %18 row_newbcast:15 row_mask:0xf bank_mask:0xf\n"
               : "+v"(ar), "+v"(ai)
               : "v"(Vr), "v"(Vi), "v"(x[0].re), "v"(x[0].im), "v"(x[1].re), "v"(x[1].im), "v"(x[2].re), "v"(x[2].im), "v"(x[3].re), "v"(x[3].im), "v"(x[4].re), "v"(x[4].im), "v"(x[5].re), "v"(x[5].im), "v"(x[6].re), "v"(x[6].im), "v"(x[7].re), "v"(x[7].im));
}
__device__ __forceinline__ void cupd_b(z64* x, double Vr, double Vi, double nr,
                                       double ni) {
  asm volatile("s_nop 1\n"
               "v_fmac_f64_dpp %0, %16, %18 row_newbcast:8 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, %16, %19 row_newbcast:8 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %0, -%17, %19 row_newbcast:8 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, %17, %18 row_newbcast:8 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %2, %16, %18 row_newbcast:9 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %3, %16, %19 row_newbcast:9 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %2, -%17, %19 row_newbcast:9 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %3, %17, %18 row_newbcast:9 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %4, %16, %18 row_newbcast:10 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %5, %16, %19 row_newbcast:10 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %4, -%17, %19 row_newbcast:10 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %5, %17, %18 row_newbcast:10 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %6, %16, %18 row_newbcast:11 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %7, %16, %19 row_newbcast:11 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %6, -%17, %19 row_newbcast:11 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %7, %17, %18 row_newbcast:11 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %8, %16, %18 row_newbcast:12 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %9, %16, %19 row_newbcast:12 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %8, -%17, %19 row_newbcast:12 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %9, %17, %18 row_newbcast:12 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %10, %16, %18 row_newbcast:13 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %11, %16, %19 row_newbcast:13 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %10, -%17, %19 row_newbcast:13 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %11, %17, %18 row_newbcast:13 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %12, %16, %18 row_newbcast:14 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %13, %16, %19 row_newbcast:14 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %12, -%17, %19 row_newbcast:14 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %13, %17, %18 row_newbcast:14 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %14, %16, %18 row_newbcast:15 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %15, %16, %19 row_newbcast:15 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %14, -%17, %19 row_newbcast:15 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %15, %17, %18 row_newbcast:15 row_mask:0xf bank_mask:0xf\n"
               : "+v"(x[0].re), "+v"(x[0].im), "+v"(x[1].re), "+v"(x[1].im), "+v"(x[2].re), "+v"(x[2].im), "+v"(x[3].re), "+v"(x[3].im), "+v"(x[4].re), "+v"(x[4].im), "+v"(x[5].re), "+v"(x[5].im), "+v"(x[6].re), "+v"(x[6].im), "+v"(x[7].re), "+v"(x[7].im)
               : "v"(Vr), "v"(Vi), "v"(nr), "v"(ni));
}
// extra term of an odd window offset: lane 0 of the third segment
__device__ __forceinline__ void cdot_x(double& ar, double& ai, double Vr, double Vi, const z64& x) {
  asm volatile("s_nop 1\n"
               "v_fmac_f64_dpp %0, %2, %4 row_newbcast:0 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, %2, %5 row_newbcast:0 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %0, %3, %5 row_newbcast:0 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, -%3, %4 row_newbcast:0 row_mask:0xf bank_mask:0xf\n"
               : "+v"(ar), "+v"(ai)
               : "v"(Vr), "v"(Vi), "v"(x.re), "v"(x.im));
}
__device__ __forceinline__ void cupd_x(z64& x, double Vr, double Vi, double nr, double ni) {
  asm volatile("s_nop 1\n"
               "v_fmac_f64_dpp %0, %2, %4 row_newbcast:0 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, %2, %5 row_newbcast:0 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %0, -%3, %5 row_newbcast:0 row_mask:0xf bank_mask:0xf\n"
               "v_fmac_f64_dpp %1, %3, %4 row_newbcast:0 row_mask:0xf bank_mask:0xf\n"
               : "+v"(x.re), "+v"(x.im)
               : "v"(Vr), "v"(Vi), "v"(nr), "v"(ni));
}

}  // namespace ehh
