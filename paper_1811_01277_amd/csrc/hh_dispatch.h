// Launcher tables shared between the kernel translation unit and the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ehh {

using StripeLaunch = hipError_t (*)(const void* hh, const void* tau, void* Q, int64_t ldq,
                                    int64_t n, int64_t nev, hipStream_t st, int num_cu);
using RefLaunch = hipError_t (*)(const void* hh, const void* tau, void* Q, int64_t ldq,
                                 int64_t n, int64_t nev, int64_t nb, hipStream_t st);

struct StripeEntry {
  int dtype;
  int nb;
  int k;
  int occ;  // waves per SIMD the kernel is compiled for
  StripeLaunch fn;
};

const StripeEntry* stripe_table(int* size);
RefLaunch ref_launcher(int dtype);

}  // namespace ehh
