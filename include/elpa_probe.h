/*
 * elpa_probe.h -- measured peaks of the arithmetic units the back-
 * transformation kernels use, for the roofline beside the vendor figures
 * (measurement support, not part of the method).
 *
 * elpa_peak_probe: runs one kernel of independent arithmetic chains on the
 * current device and reports its rate.  kind: 0 = fp64 vector FMA
 * (v_fma_f64), 1 = fp64 MFMA 16x16x4, 2 = fp32 MFMA 16x16x4, 3 = fp32 vector
 * FMA without packed instructions.  waves_per_simd: resident waves per SIMD
 * (1..8; workgroups of 4 waves, one workgroup per CU per wave level).
 * iters: loop trips (each trip issues 8 independent FMAs per lane, or 8
 * independent MFMAs per wave).
 * Outputs: *tflops = flops / kernel time (HIP events), *ms = kernel time.
 * Synchronous; allocates and frees a small output buffer.  Returns 0,
 * ELPA_ERR_ARG (-1) for a bad kind / count / pointer, ELPA_ERR_DEVICE (-5).
 */
#ifndef ELPA_PROBE_H
#define ELPA_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

int elpa_peak_probe(int32_t kind, int32_t waves_per_simd, int64_t iters, double *tflops,
                    double *ms);

#ifdef __cplusplus
}
#endif

#endif /* ELPA_PROBE_H */
