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

}  // namespace ehh
