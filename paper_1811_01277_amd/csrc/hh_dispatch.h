// Launcher tables shared between the kernel translation unit and the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/elpa_hh.h"

namespace ehh {

// S = chase steps per tile of the diagonal schedule (0 = library choice)
using StripeLaunch = hipError_t (*)(const void* hh, const void* tau, void* Q, int64_t ldq,
                                    int64_t n, int64_t nev, int64_t S, hipStream_t st,
                                    int num_cu);
using BatchedLaunch = hipError_t (*)(const elpa_hh_problem* probs, const int64_t* idx,
                                     int64_t cnt, int64_t S, hipStream_t st, int num_cu);
using RefLaunch = hipError_t (*)(const void* hh, const void* tau, void* Q, int64_t ldq,
                                 int64_t n, int64_t nev, int64_t nb, hipStream_t st);

struct StripeEntry {
  int dtype;
  int nb;
  int k;
  int occ;  // waves per SIMD the kernel is compiled for
  StripeLaunch fn;
  BatchedLaunch batched;
};

const StripeEntry* stripe_table(int* size);
RefLaunch ref_launcher(int dtype);

}  // namespace ehh
