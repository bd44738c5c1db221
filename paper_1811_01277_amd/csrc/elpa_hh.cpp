// C ABI of the tridiagonal->band back-transformation (declared in
// include/elpa_hh.h): argument validation, plan selection and launch.
#include "../../include/elpa_hh.h"

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <utility>
#include <vector>

#include "hh_common.h"
#include "hh_dispatch.h"

namespace {

int64_t elem_size(int32_t dtype) {
  switch (dtype) {
    case ELPA_R64: return 8;
    case ELPA_R32: return 4;
    case ELPA_C64: return 16;
    default: return 0;
  }
}

const ehh::StripeEntry* find_stripe(int32_t dtype, int64_t nb, int k) {
  int cnt = 0;
  const ehh::StripeEntry* tab = ehh::stripe_table(&cnt);
  for (int i = 0; i < cnt; ++i) {
    const ehh::StripeEntry& e = tab[i];
    if (e.dtype == dtype && e.nb == nb && e.k == k) return &e;
  }
  return nullptr;
}

// Default number of fused sweeps per pass for the stripe kernel.
int default_k(int32_t dtype, int64_t nb) {
  const int pref[] = {32, 16, 8, 4};
  const int prefc[] = {4, 2};
  if (dtype == ELPA_C64) {
    for (int k : prefc)
      if (find_stripe(dtype, nb, k)) return k;
    return 0;
  }
  for (int k : pref)
    if (find_stripe(dtype, nb, k)) return k;
  return 0;
}

// Compute-unit count of the current device (cached per device id).
int device_cus() {
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (dev < 0 || dev >= 64) dev = 0;
  if (cache[dev] == 0) {
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cu <= 0)
      cu = 256;
    cache[dev] = cu;
  }
  return cache[dev];
}

bool aligned(const void* p, int64_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

int validate(int64_t n, int64_t nev, int64_t nbw, const void* hh, const void* tau, void* Q,
             int64_t ldq, int32_t dtype) {
  if (n < 0 || nev < 0 || nbw < 1) return ELPA_ERR_ARG;
  const int64_t es = elem_size(dtype);
  if (es == 0) return ELPA_ERR_DTYPE;
  if (n <= 1 || nev == 0) return ELPA_OK;
  if (ldq < n) return ELPA_ERR_ARG;
  if (!hh || !tau || !Q) return ELPA_ERR_ARG;
  // byte offsets ldq*(nev-1)+n and N_refl*nbw must fit in int64
  if (nev > 1 && ldq > (INT64_MAX / es - n) / (nev - 1)) return ELPA_ERR_ARG;
  const int64_t nr = ehh::csum(n - 1, nbw);
  if (nr > INT64_MAX / nbw / es) return ELPA_ERR_ARG;
  if (!aligned(hh, es) || !aligned(tau, es) || !aligned(Q, es)) return ELPA_ERR_ALIGN;
  return ELPA_OK;
}

}  // namespace

extern "C" {

int64_t elpa_hh_num_reflectors(int64_t n, int64_t nbw) {
  if (n < 0 || nbw < 1) return -1;
  if (n <= 1) return 0;
  return ehh::csum(n - 1, nbw);
}

int64_t elpa_hh_slot_offset(int64_t n, int64_t nbw, int64_t s) {
  if (n < 1 || nbw < 1 || s < 0 || s > n - 1) return -1;
  return ehh::slot_offset(n, nbw, s);
}

int elpa_hh_plan_supported(int64_t nbw, int32_t dtype, const elpa_hh_plan* plan) {
  if (elem_size(dtype) == 0 || nbw < 1) return 0;
  const int path = plan ? plan->path : ELPA_PATH_AUTO;
  switch (path) {
    case ELPA_PATH_AUTO:
    case ELPA_PATH_REF: return 1;
    case ELPA_PATH_STRIPE: {
      const int k = (plan && plan->k > 0) ? plan->k : default_k(dtype, nbw);
      return (k > 0 && find_stripe(dtype, nbw, k)) ? 1 : 0;
    }
    default: return 0;
  }
}

int elpa_hh_trafo_plan(int64_t n, int64_t nev, int64_t nbw, const void* hh, const void* tau,
                       void* Q, int64_t ldq, int32_t dtype, void* stream,
                       const elpa_hh_plan* plan) {
  int rc = validate(n, nev, nbw, hh, tau, Q, ldq, dtype);
  if (rc != ELPA_OK) return rc;
  if (n <= 1 || nev == 0) return ELPA_OK;
  if (plan && plan->path != ELPA_PATH_AUTO && plan->path != ELPA_PATH_REF &&
      plan->path != ELPA_PATH_STRIPE)
    return ELPA_ERR_PLAN;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  int path = plan ? plan->path : ELPA_PATH_AUTO;
  int k = (plan && plan->k > 0) ? plan->k : 0;
  const ehh::StripeEntry* se = nullptr;
  if (path == ELPA_PATH_AUTO) {
    const int kd = k ? k : default_k(dtype, nbw);
    se = kd ? find_stripe(dtype, nbw, kd) : nullptr;
    path = se ? ELPA_PATH_STRIPE : ELPA_PATH_REF;
  } else if (path == ELPA_PATH_STRIPE) {
    const int kd = k ? k : default_k(dtype, nbw);
    se = kd ? find_stripe(dtype, nbw, kd) : nullptr;
    if (!se) return ELPA_ERR_PLAN;
  }
  hipError_t err;
  if (path == ELPA_PATH_STRIPE) {
    err = se->fn(hh, tau, Q, ldq, n, nev, plan ? plan->steps : 0, st, device_cus());
  } else {
    err = ehh::ref_launcher(dtype)(hh, tau, Q, ldq, n, nev, nbw, st);
  }
  return err == hipSuccess ? ELPA_OK : ELPA_ERR_DEVICE;
}

int elpa_hh_trafo_batched(const elpa_hh_problem* probs, int64_t count, void* stream,
                          const elpa_hh_plan* plan) {
  if (count < 0 || (count > 0 && !probs)) return ELPA_ERR_ARG;
  if (plan && plan->path != ELPA_PATH_AUTO && plan->path != ELPA_PATH_REF &&
      plan->path != ELPA_PATH_STRIPE)
    return ELPA_ERR_PLAN;
  for (int64_t i = 0; i < count; ++i) {
    const elpa_hh_problem& p = probs[i];
    const int rc = validate(p.n, p.nev, p.nbw, p.hh, p.tau, p.Q, p.ldq, p.dtype);
    if (rc != ELPA_OK) return rc;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int path = plan ? plan->path : ELPA_PATH_AUTO;
  const int kreq = (plan && plan->k > 0) ? plan->k : 0;
  // group by (dtype, nbw); groups without a stripe kernel go one by one
  std::map<std::pair<int32_t, int64_t>, std::vector<int64_t>> groups;
  std::vector<int64_t> singles;
  for (int64_t i = 0; i < count; ++i) {
    const elpa_hh_problem& p = probs[i];
    if (p.n <= 1 || p.nev == 0) continue;
    const int k = kreq ? kreq : default_k(p.dtype, p.nbw);
    const bool stripe = path != ELPA_PATH_REF && k > 0 && find_stripe(p.dtype, p.nbw, k);
    if (path == ELPA_PATH_STRIPE && !stripe) return ELPA_ERR_PLAN;
    if (stripe)
      groups[{p.dtype, p.nbw}].push_back(i);
    else
      singles.push_back(i);
  }
  const int cus = count > 0 ? device_cus() : 0;
  for (auto& kv : groups) {
    const int k = kreq ? kreq : default_k(kv.first.first, kv.first.second);
    const ehh::StripeEntry* se = find_stripe(kv.first.first, kv.first.second, k);
    const hipError_t err =
        se->batched(probs, kv.second.data(), (int64_t)kv.second.size(),
                    plan ? plan->steps : 0, st, cus);
    if (err != hipSuccess) return ELPA_ERR_DEVICE;
  }
  for (int64_t i : singles) {
    const elpa_hh_problem& p = probs[i];
    const hipError_t err =
        ehh::ref_launcher(p.dtype)(p.hh, p.tau, p.Q, p.ldq, p.n, p.nev, p.nbw, st);
    if (err != hipSuccess) return ELPA_ERR_DEVICE;
  }
  return ELPA_OK;
}

int elpa_hh_trafo(int64_t n, int64_t nev, int64_t nbw, const void* hh, const void* tau, void* Q,
                  int64_t ldq, int32_t dtype, void* stream) {
  return elpa_hh_trafo_plan(n, nev, nbw, hh, tau, Q, ldq, dtype, stream, nullptr);
}

const char* elpa_strerror(int code) {
  switch (code) {
    case ELPA_OK: return "success";
    case ELPA_ERR_ARG: return "invalid argument (size, leading dimension, nbw or null pointer)";
    case ELPA_ERR_DTYPE: return "unknown element type";
    case ELPA_ERR_ALIGN: return "pointer not aligned to the element size";
    case ELPA_ERR_NOMEM: return "device workspace allocation failed";
    case ELPA_ERR_DEVICE: return "HIP launch or runtime failure";
    case ELPA_ERR_PLAN: return "explicit plan cannot run this problem";
    default: return "unknown error code";
  }
}

const char* elpa_hh_version(void) { return "elpa-hip 0.1 (gfx950)"; }

}  // extern "C"
