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
// broadcast lanes l0..l7 of one or two segments.  The extra term of an odd
// window offset is segment 2's lane-0 value against one more window row.
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

// ---------------------------------------------------------------------------
// Reflector pairs.  Two consecutive reflectors A (applied first) and B of a
// chase step start on the same window register in both lane halves, so their
// dot products run in one pass over the registers (four accumulator chains)
// and their updates in another: x += bcast(vA) nwA, then x += bcast(vB) nwB
// on every register, A's terms before B's within a block.  Only A can carry
// the extra term (it is the odd offset).
// ---------------------------------------------------------------------------
#define EHH_PDOT2(l0, l1, l2, l3, l4, l5, l6, l7) \
  EHH_F(0, 4, 8, l0) EHH_F(2, 6, 8, l0) EHH_F(1, 5, 16, l0) EHH_F(3, 7, 16, l0) \
  EHH_F(0, 4, 9, l1) EHH_F(2, 6, 9, l1) EHH_F(1, 5, 17, l1) EHH_F(3, 7, 17, l1) \
  EHH_F(0, 4, 10, l2) EHH_F(2, 6, 10, l2) EHH_F(1, 5, 18, l2) EHH_F(3, 7, 18, l2) \
  EHH_F(0, 4, 11, l3) EHH_F(2, 6, 11, l3) EHH_F(1, 5, 19, l3) EHH_F(3, 7, 19, l3) \
  EHH_F(0, 4, 12, l4) EHH_F(2, 6, 12, l4) EHH_F(1, 5, 20, l4) EHH_F(3, 7, 20, l4) \
  EHH_F(0, 4, 13, l5) EHH_F(2, 6, 13, l5) EHH_F(1, 5, 21, l5) EHH_F(3, 7, 21, l5) \
  EHH_F(0, 4, 14, l6) EHH_F(2, 6, 14, l6) EHH_F(1, 5, 22, l6) EHH_F(3, 7, 22, l6) \
  EHH_F(0, 4, 15, l7) EHH_F(2, 6, 15, l7) EHH_F(1, 5, 23, l7) EHH_F(3, 7, 23, l7)
#define EHH_PUPD2(l0, l1, l2, l3, l4, l5, l6, l7) \
  EHH_F(0, 16, 20, l0) EHH_F(8, 17, 20, l0) \
  EHH_F(1, 16, 20, l1) EHH_F(9, 17, 20, l1) \
  EHH_F(2, 16, 20, l2) EHH_F(10, 17, 20, l2) \
  EHH_F(3, 16, 20, l3) EHH_F(11, 17, 20, l3) \
  EHH_F(4, 16, 20, l4) EHH_F(12, 17, 20, l4) \
  EHH_F(5, 16, 20, l5) EHH_F(13, 17, 20, l5) \
  EHH_F(6, 16, 20, l6) EHH_F(14, 17, 20, l6) \
  EHH_F(7, 16, 20, l7) EHH_F(15, 17, 20, l7) \
  EHH_F(0, 18, 21, l0) EHH_F(8, 19, 21, l0) \
  EHH_F(1, 18, 21, l1) EHH_F(9, 19, 21, l1) \
  EHH_F(2, 18, 21, l2) EHH_F(10, 19, 21, l2) \
  EHH_F(3, 18, 21, l3) EHH_F(11, 19, 21, l3) \
  EHH_F(4, 18, 21, l4) EHH_F(12, 19, 21, l4) \
  EHH_F(5, 18, 21, l5) EHH_F(13, 19, 21, l5) \
  EHH_F(6, 18, 21, l6) EHH_F(14, 19, 21, l6) \
  EHH_F(7, 18, 21, l7) EHH_F(15, 19, 21, l7)
#define EHH_PUPD2X(l0, l1, l2, l3, l4, l5, l6, l7) \
  EHH_F(0, 17, 21, l0) EHH_F(8, 18, 21, l0) \
  EHH_F(1, 17, 21, l1) EHH_F(9, 18, 21, l1) \
  EHH_F(2, 17, 21, l2) EHH_F(10, 18, 21, l2) \
  EHH_F(3, 17, 21, l3) EHH_F(11, 18, 21, l3) \
  EHH_F(4, 17, 21, l4) EHH_F(12, 18, 21, l4) \
  EHH_F(5, 17, 21, l5) EHH_F(13, 18, 21, l5) \
  EHH_F(6, 17, 21, l6) EHH_F(14, 18, 21, l6) \
  EHH_F(7, 17, 21, l7) EHH_F(15, 18, 21, l7) \
  EHH_F(0, 19, 22, l0) EHH_F(8, 20, 22, l0) \
  EHH_F(1, 19, 22, l1) EHH_F(9, 20, 22, l1) \
  EHH_F(2, 19, 22, l2) EHH_F(10, 20, 22, l2) \
  EHH_F(3, 19, 22, l3) EHH_F(11, 20, 22, l3) \
  EHH_F(4, 19, 22, l4) EHH_F(12, 20, 22, l4) \
  EHH_F(5, 19, 22, l5) EHH_F(13, 20, 22, l5) \
  EHH_F(6, 19, 22, l6) EHH_F(14, 20, 22, l6) \
  EHH_F(7, 19, 22, l7) EHH_F(15, 20, 22, l7)
#define EHH_PDOT1(l0, l1, l2, l3, l4, l5, l6, l7) \
  EHH_F(0, 4, 6, l0) EHH_F(2, 5, 6, l0) \
  EHH_F(1, 4, 7, l1) EHH_F(3, 5, 7, l1) \
  EHH_F(0, 4, 8, l2) EHH_F(2, 5, 8, l2) \
  EHH_F(1, 4, 9, l3) EHH_F(3, 5, 9, l3) \
  EHH_F(0, 4, 10, l4) EHH_F(2, 5, 10, l4) \
  EHH_F(1, 4, 11, l5) EHH_F(3, 5, 11, l5) \
  EHH_F(0, 4, 12, l6) EHH_F(2, 5, 12, l6) \
  EHH_F(1, 4, 13, l7) EHH_F(3, 5, 13, l7)
#define EHH_PUPD1(l0, l1, l2, l3, l4, l5, l6, l7) \
  EHH_F(0, 8, 10, l0) EHH_F(1, 8, 10, l1) EHH_F(2, 8, 10, l2) EHH_F(3, 8, 10, l3) \
  EHH_F(4, 8, 10, l4) EHH_F(5, 8, 10, l5) EHH_F(6, 8, 10, l6) EHH_F(7, 8, 10, l7) \
  EHH_F(0, 9, 11, l0) EHH_F(1, 9, 11, l1) EHH_F(2, 9, 11, l2) EHH_F(3, 9, 11, l3) \
  EHH_F(4, 9, 11, l4) EHH_F(5, 9, 11, l5) EHH_F(6, 9, 11, l6) EHH_F(7, 9, 11, l7)
#define EHH_PUPD1X(l0, l1, l2, l3, l4, l5, l6, l7) \
  EHH_F(0, 9, 11, l0) EHH_F(1, 9, 11, l1) EHH_F(2, 9, 11, l2) EHH_F(3, 9, 11, l3) \
  EHH_F(4, 9, 11, l4) EHH_F(5, 9, 11, l5) EHH_F(6, 9, 11, l6) EHH_F(7, 9, 11, l7) \
  EHH_F(0, 10, 12, l0) EHH_F(1, 10, 12, l1) EHH_F(2, 10, 12, l2) EHH_F(3, 10, 12, l3) \
  EHH_F(4, 10, 12, l4) EHH_F(5, 10, 12, l5) EHH_F(6, 10, 12, l6) EHH_F(7, 10, 12, l7)

// pair dot, two segments: aA0/aA1 += vA . (x, y), aB0/aB1 += vB . (x, y)
__device__ __forceinline__ void pdot2_a(double& aA0, double& aA1, double& aB0, double& aB1,
                                        double VA0, double VA1, double VB0, double VB1,
                                        const double* x, const double* y) {
  asm volatile("s_nop 1\n" EHH_X(EHH_PDOT2, EHH_LA)
               : "+v"(aA0), "+v"(aA1), "+v"(aB0), "+v"(aB1)
               : "v"(VA0), "v"(VA1), "v"(VB0), "v"(VB1), EHH_VX8(x), EHH_VX8(y));
}
__device__ __forceinline__ void pdot2_b(double& aA0, double& aA1, double& aB0, double& aB1,
                                        double VA0, double VA1, double VB0, double VB1,
                                        double VA2, const double* x, const double* y,
                                        const double* xe) {
  asm volatile("s_nop 1\n" EHH_X(EHH_PDOT2, EHH_LB) EHH_F(0, 24, 25, 0)
               : "+v"(aA0), "+v"(aA1), "+v"(aB0), "+v"(aB1)
               : "v"(VA0), "v"(VA1), "v"(VB0), "v"(VB1), EHH_VX8(x), EHH_VX8(y), "v"(VA2),
                 "v"(xe[0]));
}
// pair update, two segments
__device__ __forceinline__ void pupd2_a(double* x, double* y, double VA0, double VA1, double VB0,
                                        double VB1, double nwA, double nwB) {
  asm volatile("s_nop 1\n" EHH_X(EHH_PUPD2, EHH_LA)
               : EHH_PX8(x), EHH_PX8(y)
               : "v"(VA0), "v"(VA1), "v"(VB0), "v"(VB1), "v"(nwA), "v"(nwB));
}
__device__ __forceinline__ void pupd2_b(double* x, double* y, double* xe, double VA0, double VA1,
                                        double VB0, double VB1, double VA2, double nwA,
                                        double nwB) {
  asm volatile("s_nop 1\n" EHH_F(16, 23, 21, 0) EHH_X(EHH_PUPD2X, EHH_LB)
               : EHH_PX8(x), EHH_PX8(y), "+v"(xe[0])
               : "v"(VA0), "v"(VA1), "v"(VB0), "v"(VB1), "v"(nwA), "v"(nwB), "v"(VA2));
}
// pair dot, one segment (accumulators alternate over the broadcast lanes)
__device__ __forceinline__ void pdot1_a(double& aA0, double& aA1, double& aB0, double& aB1,
                                        double VA0, double VB0, const double* x) {
  asm volatile("s_nop 1\n" EHH_X(EHH_PDOT1, EHH_LA)
               : "+v"(aA0), "+v"(aA1), "+v"(aB0), "+v"(aB1)
               : "v"(VA0), "v"(VB0), EHH_VX8(x));
}
__device__ __forceinline__ void pdot1_b(double& aA0, double& aA1, double& aB0, double& aB1,
                                        double VA0, double VB0, double VA2, const double* x,
                                        const double* xe) {
  asm volatile("s_nop 1\n" EHH_X(EHH_PDOT1, EHH_LB) EHH_F(0, 14, 15, 0)
               : "+v"(aA0), "+v"(aA1), "+v"(aB0), "+v"(aB1)
               : "v"(VA0), "v"(VB0), EHH_VX8(x), "v"(VA2), "v"(xe[0]));
}
// pair update, one segment
__device__ __forceinline__ void pupd1_a(double* x, double VA0, double VB0, double nwA,
                                        double nwB) {
  asm volatile("s_nop 1\n" EHH_X(EHH_PUPD1, EHH_LA)
               : EHH_PX8(x)
               : "v"(VA0), "v"(VB0), "v"(nwA), "v"(nwB));
}
__device__ __forceinline__ void pupd1_b(double* x, double* xe, double VA0, double VB0, double VA2,
                                        double nwA, double nwB) {
  asm volatile("s_nop 1\n" EHH_F(8, 13, 11, 0) EHH_X(EHH_PUPD1X, EHH_LB)
               : EHH_PX8(x), "+v"(xe[0])
               : "v"(VA0), "v"(VB0), "v"(nwA), "v"(nwB), "v"(VA2));
}

// fp32 pair blocks: the same blocks on 32-bit values (v_fmac_f32 with the
// same row_newbcast broadcast), for the single-precision split kernel.
#define EHH_G(D, S, X, L) \
  "v_fmac_f32_dpp %" #D ", %" #S ", %" #X " row_newbcast:" #L " row_mask:0xf bank_mask:0xf\n"
#define EHH_PDOT2S(l0, l1, l2, l3, l4, l5, l6, l7) \
  EHH_G(0, 4, 8, l0) EHH_G(2, 6, 8, l0) EHH_G(1, 5, 16, l0) EHH_G(3, 7, 16, l0) \
  EHH_G(0, 4, 9, l1) EHH_G(2, 6, 9, l1) EHH_G(1, 5, 17, l1) EHH_G(3, 7, 17, l1) \
  EHH_G(0, 4, 10, l2) EHH_G(2, 6, 10, l2) EHH_G(1, 5, 18, l2) EHH_G(3, 7, 18, l2) \
  EHH_G(0, 4, 11, l3) EHH_G(2, 6, 11, l3) EHH_G(1, 5, 19, l3) EHH_G(3, 7, 19, l3) \
  EHH_G(0, 4, 12, l4) EHH_G(2, 6, 12, l4) EHH_G(1, 5, 20, l4) EHH_G(3, 7, 20, l4) \
  EHH_G(0, 4, 13, l5) EHH_G(2, 6, 13, l5) EHH_G(1, 5, 21, l5) EHH_G(3, 7, 21, l5) \
  EHH_G(0, 4, 14, l6) EHH_G(2, 6, 14, l6) EHH_G(1, 5, 22, l6) EHH_G(3, 7, 22, l6) \
  EHH_G(0, 4, 15, l7) EHH_G(2, 6, 15, l7) EHH_G(1, 5, 23, l7) EHH_G(3, 7, 23, l7)
#define EHH_PUPD2S(l0, l1, l2, l3, l4, l5, l6, l7) \
  EHH_G(0, 16, 20, l0) EHH_G(8, 17, 20, l0) \
  EHH_G(1, 16, 20, l1) EHH_G(9, 17, 20, l1) \
  EHH_G(2, 16, 20, l2) EHH_G(10, 17, 20, l2) \
  EHH_G(3, 16, 20, l3) EHH_G(11, 17, 20, l3) \
  EHH_G(4, 16, 20, l4) EHH_G(12, 17, 20, l4) \
  EHH_G(5, 16, 20, l5) EHH_G(13, 17, 20, l5) \
  EHH_G(6, 16, 20, l6) EHH_G(14, 17, 20, l6) \
  EHH_G(7, 16, 20, l7) EHH_G(15, 17, 20, l7) \
  EHH_G(0, 18, 21, l0) EHH_G(8, 19, 21, l0) \
  EHH_G(1, 18, 21, l1) EHH_G(9, 19, 21, l1) \
  EHH_G(2, 18, 21, l2) EHH_G(10, 19, 21, l2) \
  EHH_G(3, 18, 21, l3) EHH_G(11, 19, 21, l3) \
  EHH_G(4, 18, 21, l4) EHH_G(12, 19, 21, l4) \
  EHH_G(5, 18, 21, l5) EHH_G(13, 19, 21, l5) \
  EHH_G(6, 18, 21, l6) EHH_G(14, 19, 21, l6) \
  EHH_G(7, 18, 21, l7) EHH_G(15, 19, 21, l7)
#define EHH_PUPD2XS(l0, l1, l2, l3, l4, l5, l6, l7) \
  EHH_G(0, 17, 21, l0) EHH_G(8, 18, 21, l0) \
  EHH_G(1, 17, 21, l1) EHH_G(9, 18, 21, l1) \
  EHH_G(2, 17, 21, l2) EHH_G(10, 18, 21, l2) \
  EHH_G(3, 17, 21, l3) EHH_G(11, 18, 21, l3) \
  EHH_G(4, 17, 21, l4) EHH_G(12, 18, 21, l4) \
  EHH_G(5, 17, 21, l5) EHH_G(13, 18, 21, l5) \
  EHH_G(6, 17, 21, l6) EHH_G(14, 18, 21, l6) \
  EHH_G(7, 17, 21, l7) EHH_G(15, 18, 21, l7) \
  EHH_G(0, 19, 22, l0) EHH_G(8, 20, 22, l0) \
  EHH_G(1, 19, 22, l1) EHH_G(9, 20, 22, l1) \
  EHH_G(2, 19, 22, l2) EHH_G(10, 20, 22, l2) \
  EHH_G(3, 19, 22, l3) EHH_G(11, 20, 22, l3) \
  EHH_G(4, 19, 22, l4) EHH_G(12, 20, 22, l4) \
  EHH_G(5, 19, 22, l5) EHH_G(13, 20, 22, l5) \
  EHH_G(6, 19, 22, l6) EHH_G(14, 20, 22, l6) \
  EHH_G(7, 19, 22, l7) EHH_G(15, 20, 22, l7)
#define EHH_PDOT1S(l0, l1, l2, l3, l4, l5, l6, l7) \
  EHH_G(0, 4, 6, l0) EHH_G(2, 5, 6, l0) \
  EHH_G(1, 4, 7, l1) EHH_G(3, 5, 7, l1) \
  EHH_G(0, 4, 8, l2) EHH_G(2, 5, 8, l2) \
  EHH_G(1, 4, 9, l3) EHH_G(3, 5, 9, l3) \
  EHH_G(0, 4, 10, l4) EHH_G(2, 5, 10, l4) \
  EHH_G(1, 4, 11, l5) EHH_G(3, 5, 11, l5) \
  EHH_G(0, 4, 12, l6) EHH_G(2, 5, 12, l6) \
  EHH_G(1, 4, 13, l7) EHH_G(3, 5, 13, l7)
#define EHH_PUPD1S(l0, l1, l2, l3, l4, l5, l6, l7) \
  EHH_G(0, 8, 10, l0) EHH_G(1, 8, 10, l1) EHH_G(2, 8, 10, l2) EHH_G(3, 8, 10, l3) \
  EHH_G(4, 8, 10, l4) EHH_G(5, 8, 10, l5) EHH_G(6, 8, 10, l6) EHH_G(7, 8, 10, l7) \
  EHH_G(0, 9, 11, l0) EHH_G(1, 9, 11, l1) EHH_G(2, 9, 11, l2) EHH_G(3, 9, 11, l3) \
  EHH_G(4, 9, 11, l4) EHH_G(5, 9, 11, l5) EHH_G(6, 9, 11, l6) EHH_G(7, 9, 11, l7)
#define EHH_PUPD1XS(l0, l1, l2, l3, l4, l5, l6, l7) \
  EHH_G(0, 9, 11, l0) EHH_G(1, 9, 11, l1) EHH_G(2, 9, 11, l2) EHH_G(3, 9, 11, l3) \
  EHH_G(4, 9, 11, l4) EHH_G(5, 9, 11, l5) EHH_G(6, 9, 11, l6) EHH_G(7, 9, 11, l7) \
  EHH_G(0, 10, 12, l0) EHH_G(1, 10, 12, l1) EHH_G(2, 10, 12, l2) EHH_G(3, 10, 12, l3) \
  EHH_G(4, 10, 12, l4) EHH_G(5, 10, 12, l5) EHH_G(6, 10, 12, l6) EHH_G(7, 10, 12, l7)

// pair dot, two segments: aA0/aA1 += vA . (x, y), aB0/aB1 += vB . (x, y)
__device__ __forceinline__ void pdot2_a(float& aA0, float& aA1, float& aB0, float& aB1,
                                        float VA0, float VA1, float VB0, float VB1,
                                        const float* x, const float* y) {
  asm volatile("s_nop 1\n" EHH_X(EHH_PDOT2S, EHH_LA)
               : "+v"(aA0), "+v"(aA1), "+v"(aB0), "+v"(aB1)
               : "v"(VA0), "v"(VA1), "v"(VB0), "v"(VB1), EHH_VX8(x), EHH_VX8(y));
}
__device__ __forceinline__ void pdot2_b(float& aA0, float& aA1, float& aB0, float& aB1,
                                        float VA0, float VA1, float VB0, float VB1,
                                        float VA2, const float* x, const float* y,
                                        const float* xe) {
  asm volatile("s_nop 1\n" EHH_X(EHH_PDOT2S, EHH_LB) EHH_G(0, 24, 25, 0)
               : "+v"(aA0), "+v"(aA1), "+v"(aB0), "+v"(aB1)
               : "v"(VA0), "v"(VA1), "v"(VB0), "v"(VB1), EHH_VX8(x), EHH_VX8(y), "v"(VA2),
                 "v"(xe[0]));
}
// pair update, two segments
__device__ __forceinline__ void pupd2_a(float* x, float* y, float VA0, float VA1, float VB0,
                                        float VB1, float nwA, float nwB) {
  asm volatile("s_nop 1\n" EHH_X(EHH_PUPD2S, EHH_LA)
               : EHH_PX8(x), EHH_PX8(y)
               : "v"(VA0), "v"(VA1), "v"(VB0), "v"(VB1), "v"(nwA), "v"(nwB));
}
__device__ __forceinline__ void pupd2_b(float* x, float* y, float* xe, float VA0, float VA1,
                                        float VB0, float VB1, float VA2, float nwA,
                                        float nwB) {
  asm volatile("s_nop 1\n" EHH_G(16, 23, 21, 0) EHH_X(EHH_PUPD2XS, EHH_LB)
               : EHH_PX8(x), EHH_PX8(y), "+v"(xe[0])
               : "v"(VA0), "v"(VA1), "v"(VB0), "v"(VB1), "v"(nwA), "v"(nwB), "v"(VA2));
}
// pair dot, one segment (accumulators alternate over the broadcast lanes)
__device__ __forceinline__ void pdot1_a(float& aA0, float& aA1, float& aB0, float& aB1,
                                        float VA0, float VB0, const float* x) {
  asm volatile("s_nop 1\n" EHH_X(EHH_PDOT1S, EHH_LA)
               : "+v"(aA0), "+v"(aA1), "+v"(aB0), "+v"(aB1)
               : "v"(VA0), "v"(VB0), EHH_VX8(x));
}
__device__ __forceinline__ void pdot1_b(float& aA0, float& aA1, float& aB0, float& aB1,
                                        float VA0, float VB0, float VA2, const float* x,
                                        const float* xe) {
  asm volatile("s_nop 1\n" EHH_X(EHH_PDOT1S, EHH_LB) EHH_G(0, 14, 15, 0)
               : "+v"(aA0), "+v"(aA1), "+v"(aB0), "+v"(aB1)
               : "v"(VA0), "v"(VB0), EHH_VX8(x), "v"(VA2), "v"(xe[0]));
}
// pair update, one segment
__device__ __forceinline__ void pupd1_a(float* x, float VA0, float VB0, float nwA,
                                        float nwB) {
  asm volatile("s_nop 1\n" EHH_X(EHH_PUPD1S, EHH_LA)
               : EHH_PX8(x)
               : "v"(VA0), "v"(VB0), "v"(nwA), "v"(nwB));
}
__device__ __forceinline__ void pupd1_b(float* x, float* xe, float VA0, float VB0, float VA2,
                                        float nwA, float nwB) {
  asm volatile("s_nop 1\n" EHH_G(8, 13, 11, 0) EHH_X(EHH_PUPD1XS, EHH_LB)
               : EHH_PX8(x), "+v"(xe[0])
               : "v"(VA0), "v"(VB0), "v"(nwA), "v"(nwB), "v"(VA2));
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
