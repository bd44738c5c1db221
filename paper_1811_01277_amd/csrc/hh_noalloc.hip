// Fixed device scratch of the allocation-free back-transformation entry point
// (elpa_hh_trafo_noalloc in include/elpa_hh.h).
//
// `scratch` is a file-scope device array: every device the library runs on
// holds its own copy (ELPA_HH_NOALLOC_SCRATCH_BYTES) from code-object load to
// process end.  In host code its name is only a stand-in for the symbol, so
// its device address is looked up once per device, with that device current,
// and only that address is ever handed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "../../include/elpa_hh.h"

static __device__ __align__(256) unsigned char scratch[ELPA_HH_NOALLOC_SCRATCH_BYTES];

namespace ehh {

// Device address of the current device's scratch (hipGetSymbolAddress on
// first use per device); *bytes = its size.
hipError_t noalloc_scratch(void** out, size_t* bytes) {
  static std::mutex mu;
  static std::vector<void*> addr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> g(mu);
  if ((size_t)dev >= addr.size()) addr.resize((size_t)dev + 1, nullptr);
  if (!addr[(size_t)dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return e != hipSuccess ? e : hipErrorInvalidSymbol;
    }
    addr[(size_t)dev] = p;
  }
  *out = addr[(size_t)dev];
  *bytes = sizeof(scratch);
  return hipSuccess;
}

}  // namespace ehh
