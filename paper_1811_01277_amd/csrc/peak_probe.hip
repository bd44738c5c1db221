// Arithmetic-unit peak probes (include/elpa_probe.h): independent FMA or MFMA
// chains in a loop, as many waves per SIMD as asked, timed with HIP events.
#include <hip/hip_runtime.h>

#include "../../include/elpa_hh.h"
#include "../../include/elpa_probe.h"

namespace {

typedef double p_d4 __attribute__((ext_vector_type(4)));
typedef float p_f4 __attribute__((ext_vector_type(4)));

template <typename T>
__global__ __launch_bounds__(256) void k_probe_fma(T* __restrict__ out, int64_t iters, T a, T b) {
  T acc[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) acc[i] = (T)(threadIdx.x + i);
  for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = __builtin_fma(acc[i], a, b);
  }
  T s = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) s += acc[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

template <>
__global__ __launch_bounds__(256) void k_probe_fma<float>(float* __restrict__ out, int64_t iters,
                                                          float a, float b) {
  float acc[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) acc[i] = (float)(threadIdx.x + i);
  for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = __builtin_fmaf(acc[i], a, b);
  }
  float s = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) s += acc[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_probe_mfma64(double* __restrict__ out, int64_t iters,
                                                      double a, double b) {
  p_d4 acc[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) acc[i] = p_d4{(double)i, 0.0, 0.0, 0.0};
  const double x = a + threadIdx.x, y = b - threadIdx.x;
  for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, acc[i], 0, 0, 0);
  }
  double s = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_probe_mfma32(float* __restrict__ out, int64_t iters,
                                                      float a, float b) {
  p_f4 acc[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) acc[i] = p_f4{(float)i, 0.f, 0.f, 0.f};
  const float x = a + threadIdx.x, y = b - threadIdx.x;
  for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, acc[i], 0, 0, 0);
  }
  float s = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

extern "C" int elpa_peak_probe(int32_t kind, int32_t waves_per_simd, int64_t iters,
                               double* tflops, double* ms) {
  if (kind < 0 || kind > 3 || waves_per_simd < 1 || waves_per_simd > 8 || iters < 1 || !tflops ||
      !ms)
    return ELPA_ERR_ARG;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return ELPA_ERR_DEVICE;
  const unsigned blocks = (unsigned)(cus * waves_per_simd);  // 4 waves each: one per SIMD
  const size_t threads = (size_t)blocks * 256;
  void* out = nullptr;
  if (hipMalloc(&out, threads * sizeof(double)) != hipSuccess) return ELPA_ERR_DEVICE;
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  auto launch = [&](int64_t n) {
    switch (kind) {
      case 0: hipLaunchKernelGGL(k_probe_fma<double>, dim3(blocks), dim3(256), 0, 0, (double*)out, n, 0.999, 1e-3); break;
      case 1: hipLaunchKernelGGL(k_probe_mfma64, dim3(blocks), dim3(256), 0, 0, (double*)out, n, 1e-3, 1e-3); break;
      case 2: hipLaunchKernelGGL(k_probe_mfma32, dim3(blocks), dim3(256), 0, 0, (float*)out, n, 1e-3f, 1e-3f); break;
      default: hipLaunchKernelGGL(k_probe_fma<float>, dim3(blocks), dim3(256), 0, 0, (float*)out, n, 0.999f, 1e-3f); break;
    }
  };
  if (e == hipSuccess) {
    launch(iters);  // warm-up (also brings the clocks up)
    launch(iters);
    e = hipEventRecord(a, 0);
  }
  if (e == hipSuccess) {
    launch(iters);
    e = hipEventRecord(b, 0);
  }
  if (e == hipSuccess) e = hipEventSynchronize(b);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  (void)hipFree(out);
  if (e != hipSuccess || t <= 0.f) return ELPA_ERR_DEVICE;
  // flops per lane-trip: 8 FMAs x 2; per wave-trip: 8 MFMAs of 16x16x4 (2048 flops each)
  const double waves = (double)threads / 64.0;
  const double fl = (kind == 0 || kind == 3) ? (double)threads * (double)iters * 16.0
                                             : waves * (double)iters * 8.0 * 2048.0;
  *ms = t;
  *tflops = fl / (t * 1e-3) / 1e12;
  return ELPA_OK;
}
