// C ABI of the tridiagonal->band back-transformation (declared in
// include/elpa_hh.h): argument validation, plan selection and launch.
#include "../../include/elpa_hh.h"

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
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

const ehh::StripeEntry* find_entry(int path, int32_t dtype, int64_t nb, int k) {
  int cnt = 0;
  const ehh::StripeEntry* tab = path == ELPA_PATH_SPLIT ? ehh::split_table(&cnt)
                                : path == ELPA_PATH_WY  ? ehh::wy_table(&cnt)
                                                        : ehh::stripe_table(&cnt);
  for (int i = 0; i < cnt; ++i) {
    const ehh::StripeEntry& e = tab[i];
    if (e.path == path && e.dtype == dtype && e.nb == nb && e.k == k) return &e;
  }
  return nullptr;
}

// Library default of the sweeps fused per pass, per kernel family: the first
// compiled entry in order of preference (0 if none).
int default_k(int path, int32_t dtype, int64_t nb, bool batched) {
  static const int split_pref[] = {80, 64, 48, 32, 96, 24, 16};
  // batched calls at nbw = 32: the widest k that holds its window without
  // spilling (k = 96 takes the 256-problem batched workload from 42.2 to
  // 39.4 ms of kernel time against k = 64; a single small problem has too
  // few sweep blocks for it: n = 512 takes 0.50 instead of 0.43 ms)
  static const int split_pref32[] = {96, 64, 48, 32};
  static const int wy_pref[] = {160, 128, 96, 64, 48, 32};
  static const int wy_pref32[] = {96, 64, 32, 128};
  static const int wy_pref_c[] = {48, 32, 16};
  static const int stripe_pref[] = {32, 16, 8, 4};
  static const int stripe_pref_c[] = {4, 2};
  if (path == ELPA_PATH_SPLIT) {
    if (nb == 32 && batched)
      for (int k : split_pref32)
        if (find_entry(path, dtype, nb, k)) return k;
    for (int k : split_pref)
      if (find_entry(path, dtype, nb, k)) return k;
    return 0;
  }
  if (path == ELPA_PATH_WY) {
    const int* pref = dtype == ELPA_C64 ? wy_pref_c : dtype == ELPA_R32 ? wy_pref32 : wy_pref;
    const int cnt = dtype == ELPA_C64 ? 3 : dtype == ELPA_R32 ? 4 : 6;
    for (int i = 0; i < cnt; ++i)
      if (find_entry(path, dtype, nb, pref[i])) return pref[i];
    return 0;
  }
  if (dtype == ELPA_C64) {
    for (int k : stripe_pref_c)
      if (find_entry(path, dtype, nb, k)) return k;
    return 0;
  }
  for (int k : stripe_pref)
    if (find_entry(path, dtype, nb, k)) return k;
  return 0;
}

// Library choice for a single problem of size n with semi-bandwidth 64, from
// sweeps over n = 1000 .. 20000 (nev = n) on this GPU: the compact-WY MFMA
// kernel for fp32 (k = 96, from n = 6000 k = 160) and complex fp64 (k = 48)
// at every size, and for fp64 from n = 3000 on (k = 128, from n = 6000
// k = 160): a larger k reuses every loaded row more but leaves fewer sweep
// blocks to run side by side (fp32 at n = 20000: 82.2 TFLOP/s at k = 160,
// 77.3 at 96; at n = 4000: 36.9 against 39.2);
// 0 = the two-lane VALU kernel (fp64 below n = 3000, complex at nbw = 32,
// other nbw, batched calls).  fp64 with fewer than 1024 columns
// also takes the two-lane kernel:
// the compact-WY kernel's T-build, which does not shrink with nev, is then a
// large part of the call (n = 8192, nev = 819: 6.7 ms two-lane, 7.9 ms WY;
// nev = 2000 at n = 20000 is faster on WY).  nev = 0: not known, taken as
// large.
int auto_wy_k(int32_t dtype, int64_t nb, int64_t n, int64_t nev) {
  // nbw = 32, real: the compact-WY kernel from n = 2000 despite its 1.5x
  // executed flops there (fp64, n = 2000 / 4000 / 6000 / 12000: 8.0 / 21.7 /
  // 29.2 / 34.3 TFLOP/s against 6.1 / 17.1 / 25.1 / 31.7 for the two-lane
  // kernel; fp32 at n = 2000 / 6000 / 12000: 10.6 / 44.3 / 54.4 against 7.3 /
  // 36.8 / 52.6); complex keeps the two-lane kernel (n = 6000: 37.5 against
  // 31.4 for WY k = 32)
  if (nb == 32)
    return ((dtype == ELPA_R64 || dtype == ELPA_R32) && n >= 2000 &&
            (nev == 0 || nev >= 1024))
               ? 96
               : 0;
  if (nb != 64) return 0;
  if (dtype == ELPA_R32) return n >= 6000 ? 160 : 96;
  if (dtype == ELPA_C64) return 48;
  if (dtype == ELPA_R64 && n >= 3000 && (nev == 0 || nev >= 1024)) return n >= 6000 ? 160 : 128;
  return 0;
}

// Kernel that runs (dtype, nb) of size n under `plan` (NULL = library
// choice).  Returns the table entry, or nullptr with *path = ELPA_PATH_REF for
// the reference kernel; *rc = ELPA_ERR_PLAN if an explicit plan cannot run.
// batched: the kernel must have a batched form, and the library choice
// prefers the two-lane kernel (its one-launch batched schedule).
const ehh::StripeEntry* resolve(int32_t dtype, int64_t nb, const elpa_hh_plan* plan, int* path,
                                int* rc, bool batched = false, int64_t n = 0, int64_t nev = 0) {
  *rc = ELPA_OK;
  if (plan && (plan->order < ELPA_ORDER_AUTO || plan->order > ELPA_ORDER_XCD ||
               plan->streams < 0 || plan->streams > 8 || plan->batch < ELPA_BATCH_AUTO ||
               plan->batch > ELPA_BATCH_DIAGONAL)) {
    *rc = ELPA_ERR_PLAN;
    return nullptr;
  }
  const int want = plan ? plan->path : ELPA_PATH_AUTO;
  const int k = (plan && plan->k > 0) ? plan->k : 0;
  *path = ELPA_PATH_REF;
  switch (want) {
    case ELPA_PATH_REF: return nullptr;
    case ELPA_PATH_STRIPE:
    case ELPA_PATH_SPLIT:
    case ELPA_PATH_WY: {
      const int kk = k ? k : default_k(want, dtype, nb, batched);
      const ehh::StripeEntry* e = kk ? find_entry(want, dtype, nb, kk) : nullptr;
      if (!e || (batched && !e->batched)) {
        *rc = ELPA_ERR_PLAN;
        return nullptr;
      }
      *path = want;
      return e;
    }
    case ELPA_PATH_AUTO: {
      if (!batched && k == 0) {
        const int wk = auto_wy_k(dtype, nb, n, nev);
        const ehh::StripeEntry* e = wk ? find_entry(ELPA_PATH_WY, dtype, nb, wk) : nullptr;
        if (e) {
          *path = ELPA_PATH_WY;
          return e;
        }
      }
      // the two-lane VALU kernel where one is compiled (fp64, fp32 and
      // complex), then for fp32 the compact-WY MFMA path, then the one-lane
      // kernel
      const int order32[] = {ELPA_PATH_SPLIT, ELPA_PATH_WY, ELPA_PATH_STRIPE};
      const int order[] = {ELPA_PATH_SPLIT, ELPA_PATH_STRIPE};
      const int* fams = dtype == ELPA_R32 ? order32 : order;
      const int nf = dtype == ELPA_R32 ? 3 : 2;
      for (int f = 0; f < nf; ++f) {
        const int fam = fams[f];
        const int kk = k ? k : default_k(fam, dtype, nb, batched);
        const ehh::StripeEntry* e = kk ? find_entry(fam, dtype, nb, kk) : nullptr;
        if (e && !(batched && !e->batched)) {
          *path = fam;
          return e;
        }
      }
      return nullptr;
    }
    default: *rc = ELPA_ERR_PLAN; return nullptr;
  }
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

// The plan a call runs.  A plan that leaves the kernel open (path AUTO, k,
// steps and batch 0; NULL included) takes the tuner's plan for the size
// class of (n, nev) if there is one, with the caller's order and streams
// where those are set; otherwise the caller's plan (NULL: library choice).
const elpa_hh_plan* effective_plan(int32_t dtype, int64_t nbw, int64_t n, int64_t nev,
                                   const elpa_hh_plan* plan, elpa_hh_plan* buf) {
  const bool open = !plan || (plan->path == ELPA_PATH_AUTO && plan->k == 0 &&
                              plan->steps == 0 && plan->batch == 0);
  if (!open || !ehh::tuner_lookup(dtype, nbw, n, nev, buf)) return plan;
  if (plan && plan->order != 0) buf->order = plan->order;
  if (plan && plan->streams != 0) buf->streams = plan->streams;
  return buf;
}

// Tile options of a plan (NULL = library choice).
ehh::TileOpts tile_opts(const elpa_hh_plan* plan) {
  ehh::TileOpts o{};
  o.steps = plan ? plan->steps : 0;
  o.xcd = (plan && plan->order == ELPA_ORDER_XCD) ? 8 : 1;
  // two stripe groups by default: one group's launch tails overlap the other's
  o.streams = (plan && plan->streams > 0) ? plan->streams : 2;
  o.batch = plan ? plan->batch : ELPA_BATCH_AUTO;
  o.order = plan ? plan->order : ELPA_ORDER_AUTO;
  return o;
}

// Status code of a launcher's HIP result.
int status_of(hipError_t e) {
  return e == hipSuccess ? ELPA_OK : (e == hipErrorOutOfMemory ? ELPA_ERR_NOMEM : ELPA_ERR_DEVICE);
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

// A new call: forget the previous call's events.
void prof_begin_call(int path) {
  ehh::ProfState& p = ehh::prof_state();
  if (!p.on) return;
  p.started = p.recorded = false;
  p.launches = 0;
  p.path = path;
  p.k = 0;
  p.steps = 0;
  p.streams = 1;
}

}  // namespace

// A prepared batched call: per kernel group its device workspace and tables;
// problems of the reference kernel, which needs none, are kept as arguments.
struct elpa_hh_batch {
  int dev = -1;
  int path = ELPA_PATH_AUTO;  // reported by the profile when there is one group
  std::vector<std::unique_ptr<ehh::PreparedGroup>> groups;
  std::vector<elpa_hh_problem> singles;
};

namespace {

// One problem prepared as the single-problem call: the kernel the library
// picks for a single call on a workspace allocated once.
class SinglePrepared : public ehh::PreparedGroup {
 public:
  SinglePrepared(const elpa_hh_problem& p, const ehh::StripeEntry* se, ehh::TileOpts opt,
                 int num_cu)
      : p_(p), se_(se), opt_(opt), num_cu_(num_cu) {}
  ~SinglePrepared() override {
    if (ws_) (void)hipFree(ws_);
  }
  hipError_t init() {
    bytes_ = se_->workspace(p_.n, p_.nev);
    if (bytes_ == 0) return hipSuccess;
    const hipError_t err = hipMalloc(&ws_, bytes_);
    if (err != hipSuccess) {
      ws_ = nullptr;
      (void)hipGetLastError();
    }
    return err;
  }
  hipError_t run(hipStream_t st) override {
    return se_->with_ws(p_.hh, p_.tau, p_.Q, p_.ldq, p_.n, p_.nev, opt_, st, num_cu_, ws_);
  }
  size_t bytes() const override { return bytes_; }

 private:
  elpa_hh_problem p_;
  const ehh::StripeEntry* se_;
  ehh::TileOpts opt_;
  int num_cu_;
  void* ws_ = nullptr;
  size_t bytes_ = 0;
};

}  // namespace

namespace ehh {
ProfState& prof_state() {
  static thread_local ProfState s;
  return s;
}
}  // namespace ehh

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
  int path = 0, rc = 0;
  (void)resolve(dtype, nbw, plan, &path, &rc);
  return rc == ELPA_OK ? 1 : 0;
}

int elpa_hh_chosen_plan(int64_t n, int64_t nev, int64_t nbw, int32_t dtype, int32_t batched,
                        const elpa_hh_plan* plan, elpa_hh_plan* out) {
  if (!out || n < 0 || nev < 0 || nbw < 1) return ELPA_ERR_ARG;
  if (elem_size(dtype) == 0) return ELPA_ERR_DTYPE;
  elpa_hh_plan tuned{};
  const elpa_hh_plan* pp = effective_plan(dtype, nbw, n, nev, plan, &tuned);
  int path = 0, rc = 0;
  const ehh::StripeEntry* se = resolve(dtype, nbw, pp, &path, &rc, batched != 0, n, nev);
  if (rc != ELPA_OK) return rc;
  *out = pp ? *pp : elpa_hh_plan{};
  out->path = path;
  out->k = se ? se->k : 0;
  return ELPA_OK;
}

int elpa_hh_trafo_plan(int64_t n, int64_t nev, int64_t nbw, const void* hh, const void* tau,
                       void* Q, int64_t ldq, int32_t dtype, void* stream,
                       const elpa_hh_plan* plan) {
  int rc = validate(n, nev, nbw, hh, tau, Q, ldq, dtype);
  if (rc != ELPA_OK) return rc;
  elpa_hh_plan tuned{};
  plan = effective_plan(dtype, nbw, n, nev, plan, &tuned);
  int path = 0;
  const ehh::StripeEntry* se = resolve(dtype, nbw, plan, &path, &rc, false, n, nev);
  if (rc != ELPA_OK) return rc;
  if (n <= 1 || nev == 0) return ELPA_OK;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  prof_begin_call(path);
  hipError_t err;
  if (se) {
    err = se->fn(hh, tau, Q, ldq, n, nev, tile_opts(plan), st, device_cus());
  } else {
    ehh::ProfScope prof(st, 0, 0);
    prof.before(st);
    err = ehh::ref_launcher(dtype)(hh, tau, Q, ldq, n, nev, nbw, st);
    prof.after(st);
  }
  return status_of(err);
}

int elpa_hh_trafo_batched(const elpa_hh_problem* probs, int64_t count, void* stream,
                          const elpa_hh_plan* plan) {
  if (count < 0 || (count > 0 && !probs)) return ELPA_ERR_ARG;
  if (plan && (plan->path < ELPA_PATH_AUTO || plan->path > ELPA_PATH_WY)) return ELPA_ERR_PLAN;
  for (int64_t i = 0; i < count; ++i) {
    const elpa_hh_problem& p = probs[i];
    const int rc = validate(p.n, p.nev, p.nbw, p.hh, p.tau, p.Q, p.ldq, p.dtype);
    if (rc != ELPA_OK) return rc;
  }
  // group by (dtype, nbw): one launch sequence per group with a stripe kernel,
  // the reference kernel one problem at a time otherwise
  // problems that run the same kernel (a tuned plan may pick another k for
  // another size class) share one launch sequence, in order of first use
  std::vector<const ehh::StripeEntry*> order;
  std::map<const ehh::StripeEntry*, std::vector<int64_t>> groups;
  std::vector<int64_t> singles;
  int last_path = ELPA_PATH_REF;
  for (int64_t i = 0; i < count; ++i) {
    const elpa_hh_problem& p = probs[i];
    elpa_hh_plan tuned{};
    const elpa_hh_plan* pp = effective_plan(p.dtype, p.nbw, p.n, p.nev, plan, &tuned);
    int path = 0, rc = 0;
    const ehh::StripeEntry* se = resolve(p.dtype, p.nbw, pp, &path, &rc, true);
    if (rc != ELPA_OK) return rc;
    if (p.n <= 1 || p.nev == 0) continue;
    last_path = path;
    if (se) {
      if (!groups.count(se)) order.push_back(se);
      groups[se].push_back(i);
    } else {
      singles.push_back(i);
    }
  }
  if (groups.empty() && singles.empty()) return ELPA_OK;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  prof_begin_call(groups.size() + singles.size() == 1 ? last_path : ELPA_PATH_AUTO);
  const int cus = device_cus();
  for (const ehh::StripeEntry* se : order) {
    const std::vector<int64_t>& ids = groups[se];
    const hipError_t err = se->batched(probs, ids.data(), (int64_t)ids.size(),
                                       tile_opts(plan), st, cus);
    if (err != hipSuccess) return status_of(err);
  }
  for (int64_t i : singles) {
    const elpa_hh_problem& p = probs[i];
    ehh::ProfScope prof(st, 0, 0);
    prof.before(st);
    const hipError_t err =
        ehh::ref_launcher(p.dtype)(p.hh, p.tau, p.Q, p.ldq, p.n, p.nev, p.nbw, st);
    prof.after(st);
    if (err != hipSuccess) return status_of(err);
  }
  return ELPA_OK;
}

int elpa_hh_batch_create(const elpa_hh_problem* probs, int64_t count, const elpa_hh_plan* plan,
                         elpa_hh_batch** out) {
  if (!out) return ELPA_ERR_ARG;
  *out = nullptr;
  if (count < 0 || (count > 0 && !probs)) return ELPA_ERR_ARG;
  if (plan && (plan->path < ELPA_PATH_AUTO || plan->path > ELPA_PATH_WY)) return ELPA_ERR_PLAN;
  for (int64_t i = 0; i < count; ++i) {
    const elpa_hh_problem& p = probs[i];
    const int rc = validate(p.n, p.nev, p.nbw, p.hh, p.tau, p.Q, p.ldq, p.dtype);
    if (rc != ELPA_OK) return rc;
  }
  // the same grouping as elpa_hh_trafo_batched; every group needs a prepared form
  std::vector<const ehh::StripeEntry*> order;
  std::map<const ehh::StripeEntry*, std::vector<int64_t>> groups;
  auto b = std::make_unique<elpa_hh_batch>();
  if (hipGetDevice(&b->dev) != hipSuccess) return ELPA_ERR_DEVICE;
  const int cus = device_cus();
  // one problem with work: the kernel and plan of the single-problem call
  int64_t live = 0, one = -1;
  for (int64_t i = 0; i < count; ++i)
    if (probs[i].n > 1 && probs[i].nev > 0) ++live, one = i;
  if (live == 1) {
    const elpa_hh_problem& p = probs[one];
    elpa_hh_plan tuned{};
    const elpa_hh_plan* pp = effective_plan(p.dtype, p.nbw, p.n, p.nev, plan, &tuned);
    int path = 0, rc = 0;
    const ehh::StripeEntry* se = resolve(p.dtype, p.nbw, pp, &path, &rc, false, p.n, p.nev);
    if (rc != ELPA_OK) return rc;
    // every problem's plan must resolve, as in the batched call
    for (int64_t i = 0; i < count; ++i) {
      if (i == one) continue;
      elpa_hh_plan t2{};
      const elpa_hh_plan* p2 =
          effective_plan(probs[i].dtype, probs[i].nbw, probs[i].n, probs[i].nev, plan, &t2);
      int path2 = 0;
      (void)resolve(probs[i].dtype, probs[i].nbw, p2, &path2, &rc, true);
      if (rc != ELPA_OK) return rc;
    }
    b->path = path;
    if (!se) {
      b->singles.push_back(p);
    } else if (se->with_ws) {
      auto g = std::make_unique<SinglePrepared>(p, se, tile_opts(pp), cus);
      const hipError_t err = g->init();
      if (err != hipSuccess) return status_of(err);
      b->groups.emplace_back(std::move(g));
    } else {
      return ELPA_ERR_PLAN;
    }
    *out = b.release();
    return ELPA_OK;
  }
  int last_path = ELPA_PATH_REF;
  for (int64_t i = 0; i < count; ++i) {
    const elpa_hh_problem& p = probs[i];
    elpa_hh_plan tuned{};
    const elpa_hh_plan* pp = effective_plan(p.dtype, p.nbw, p.n, p.nev, plan, &tuned);
    int path = 0, rc = 0;
    const ehh::StripeEntry* se = resolve(p.dtype, p.nbw, pp, &path, &rc, true);
    if (rc != ELPA_OK) return rc;
    if (p.n <= 1 || p.nev == 0) continue;
    last_path = path;
    if (se) {
      if (!se->prepare) return ELPA_ERR_PLAN;
      if (!groups.count(se)) order.push_back(se);
      groups[se].push_back(i);
    } else {
      b->singles.push_back(p);
    }
  }
  b->path = groups.size() + b->singles.size() == 1 ? last_path : ELPA_PATH_AUTO;
  for (const ehh::StripeEntry* se : order) {
    const std::vector<int64_t>& ids = groups[se];
    ehh::PreparedGroup* g = nullptr;
    const hipError_t err = se->prepare(probs, ids.data(), (int64_t)ids.size(), tile_opts(plan),
                                       cus, &g);
    if (err != hipSuccess) return status_of(err);
    b->groups.emplace_back(g);
  }
  *out = b.release();
  return ELPA_OK;
}

int elpa_hh_batch_run(elpa_hh_batch* b, void* stream) {
  if (!b) return ELPA_ERR_ARG;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return ELPA_ERR_DEVICE;
  if (dev != b->dev) return ELPA_ERR_ARG;
  if (b->groups.empty() && b->singles.empty()) return ELPA_OK;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  prof_begin_call(b->path);
  for (auto& g : b->groups) {
    const hipError_t err = g->run(st);
    if (err != hipSuccess) return status_of(err);
  }
  for (const elpa_hh_problem& p : b->singles) {
    ehh::ProfScope prof(st, 0, 0);
    prof.before(st);
    const hipError_t err =
        ehh::ref_launcher(p.dtype)(p.hh, p.tau, p.Q, p.ldq, p.n, p.nev, p.nbw, st);
    prof.after(st);
    if (err != hipSuccess) return status_of(err);
  }
  return ELPA_OK;
}

int64_t elpa_hh_batch_bytes(const elpa_hh_batch* b) {
  if (!b) return -1;
  int64_t s = 0;
  for (const auto& g : b->groups) s += (int64_t)g->bytes();
  return s;
}

int elpa_hh_batch_destroy(elpa_hh_batch* b) {
  if (!b) return ELPA_OK;
  int cur = -1;
  const bool switch_dev = hipGetDevice(&cur) == hipSuccess && cur != b->dev && b->dev >= 0;
  if (switch_dev) (void)hipSetDevice(b->dev);
  delete b;
  if (switch_dev) (void)hipSetDevice(cur);
  return ELPA_OK;
}

int elpa_hh_trafo(int64_t n, int64_t nev, int64_t nbw, const void* hh, const void* tau, void* Q,
                  int64_t ldq, int32_t dtype, void* stream) {
  return elpa_hh_trafo_plan(n, nev, nbw, hh, tau, Q, ldq, dtype, stream, nullptr);
}

int elpa_hh_trafo_noalloc(int64_t n, int64_t nev, int64_t nbw, const void* hh, const void* tau,
                          void* Q, int64_t ldq, int32_t dtype, void* stream) {
  int rc = validate(n, nev, nbw, hh, tau, Q, ldq, dtype);
  if (rc != ELPA_OK) return rc;
  if (n <= 1 || nev == 0) return ELPA_OK;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  // the library's default two-lane kernel, one stripe group on the caller's
  // stream; no tuner lookup (a tuned plan may name a family without a
  // caller-workspace form)
  const elpa_hh_plan split{ELPA_PATH_SPLIT, 0, 0, 0, 1, 0};
  int path = 0;
  const ehh::StripeEntry* se = resolve(dtype, nbw, &split, &path, &rc);
  // no timing events are created or recorded on this path
  ehh::ProfState& prof = ehh::prof_state();
  const bool prof_on = prof.on;
  prof.on = false;
  hipError_t err;
  if (rc != ELPA_OK || !se || !se->with_ws) {
    // no two-lane kernel for this nbw: the reference kernel works in place
    err = ehh::ref_launcher(dtype)(hh, tau, Q, ldq, n, nev, nbw, st);
  } else {
    void* ws = nullptr;
    size_t cap = 0;
    err = ehh::noalloc_scratch(&ws, &cap);
    if (err == hipSuccess && se->workspace(n, nev) > cap) {
      prof.on = prof_on;
      return ELPA_ERR_ADMIT;
    }
    if (err == hipSuccess)
      err = se->with_ws(hh, tau, Q, ldq, n, nev, tile_opts(&split), st, device_cus(), ws);
  }
  prof.on = prof_on;
  return status_of(err);
}

int64_t elpa_hh_workspace_bytes(int64_t n, int64_t nev, int64_t nbw, int32_t dtype,
                                const elpa_hh_plan* plan) {
  if (n < 0 || nev < 0 || nbw < 1 || elem_size(dtype) == 0) return -1;
  elpa_hh_plan tuned{};
  plan = effective_plan(dtype, nbw, n, nev, plan, &tuned);
  int path = 0, rc = 0;
  const ehh::StripeEntry* se = resolve(dtype, nbw, plan, &path, &rc, false, n, nev);
  if (rc != ELPA_OK) return -1;
  if (n <= 1 || nev == 0 || !se) return 0;
  return (int64_t)se->workspace(n, nev);
}

int64_t elpa_hh_workspace_bytes_batched(const elpa_hh_problem* probs, int64_t count,
                                        const elpa_hh_plan* plan) {
  if (count < 0 || (count > 0 && !probs)) return -1;
  int64_t total = 0, launches = 0, groups = 0, units = 0;
  for (int64_t i = 0; i < count; ++i) {
    const elpa_hh_problem& p = probs[i];
    if (p.n < 0 || p.nev < 0 || p.nbw < 1 || elem_size(p.dtype) == 0) return -1;
    elpa_hh_plan tuned{};
    const elpa_hh_plan* pp = effective_plan(p.dtype, p.nbw, p.n, p.nev, plan, &tuned);
    int path = 0, rc = 0;
    const ehh::StripeEntry* se = resolve(p.dtype, p.nbw, pp, &path, &rc, true);
    if (rc != ELPA_OK) return -1;
    if (p.n <= 1 || p.nev == 0 || !se) continue;
    total += (int64_t)se->workspace(p.n, p.nev);
    ++groups;
    // schedule entries: at most one per problem and launch (S >= 1)
    launches += (p.n - 1 + se->k - 1) / se->k + (p.n - 1 + p.nbw - 1) / p.nbw;
    units += (p.nev + 15) / 16;  // stripes (at least 16 columns each)
  }
  if (groups == 0) return 0;
  const int64_t desc = 256;  // generous bound of one descriptor / entry
  // one-launch unit map: at most 8 ids (one per die) per stripe, 4 bytes each
  return total + (groups + launches) * desc + units * 32 + 4096;
}

int elpa_hh_profile_enable(int on) {
  ehh::ProfState& p = ehh::prof_state();
  if (p.a) (void)hipEventDestroy(p.a);
  if (p.b) (void)hipEventDestroy(p.b);
  for (hipEvent_t e : p.ev) (void)hipEventDestroy(e);
  p = ehh::ProfState{};
  if (!on) return ELPA_OK;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return ELPA_ERR_DEVICE;
  if (hipEventCreate(&p.a) != hipSuccess || hipEventCreate(&p.b) != hipSuccess) {
    if (p.a) (void)hipEventDestroy(p.a);
    p = ehh::ProfState{};
    return ELPA_ERR_DEVICE;
  }
  p.dev = dev;
  p.on = true;
  return ELPA_OK;
}

int elpa_hh_profile_last(elpa_hh_profile* out) {
  ehh::ProfState& p = ehh::prof_state();
  if (!out || !p.on || !p.recorded) return ELPA_ERR_ARG;
  float ms = 0.f;
  if (hipEventSynchronize(p.b) != hipSuccess || hipEventElapsedTime(&ms, p.a, p.b) != hipSuccess)
    return ELPA_ERR_DEVICE;
  double sum = 0.0;
  for (int64_t i = 0; i < p.launches; ++i) {
    float d = 0.f;
    if (hipEventElapsedTime(&d, p.ev[2 * (size_t)i], p.ev[2 * (size_t)i + 1]) != hipSuccess)
      return ELPA_ERR_DEVICE;
    sum += d;
  }
  out->kernel_ms = ms;
  out->launches = p.launches;
  out->path = p.path;
  out->k = p.k;
  out->steps = p.steps;
  out->sum_launch_ms = sum;
  out->streams = p.streams;
  out->reserved = 0;
  return ELPA_OK;
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
    case ELPA_ERR_ADMIT:
      return "the problem's workspace exceeds the fixed scratch of the allocation-free entry point";
    default: return "unknown error code";
  }
}

const char* elpa_hh_version(void) { return "elpa-hip 0.2 (gfx950)"; }

}  // extern "C"
