// Plan tuner of the tridiagonal->band back-transformation (C ABI in
// include/elpa_hh.h): a per-process cache of measured plans keyed by
// (element type, nbw, size class of n, size class of nev), the measurement
// that fills it, and its text save / load.
//
// The tuned parameters are the kernel family (one-lane stripe, two-lane
// stripe, compact-WY MFMA), the sweeps fused per pass k (the reflector
// grouping), the chase steps per tile (the stripe tile height) and the number
// of stripe-group streams.  Calls without an explicit plan use the cached
// plan of their size class when there is one.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <tuple>
#include <vector>

#include "../../include/elpa_hh.h"
#include "hh_dispatch.h"

namespace ehh {

namespace {

// size class: quarter octaves (sizes within ~19 % share a class)
int64_t size_class(int64_t x) {
  if (x < 1) return 0;
  return (int64_t)std::floor(4.0 * std::log2((double)x) + 1e-9);
}

using Key = std::tuple<int32_t, int64_t, int64_t, int64_t>;

struct Cache {
  std::mutex mu;
  std::map<Key, elpa_hh_plan> plans;
  static Cache& get() {
    static Cache c;
    return c;
  }
};

Key key_of(int32_t dtype, int64_t nbw, int64_t n, int64_t nev) {
  return Key{dtype, nbw, size_class(n), size_class(nev)};
}

bool plan_valid(const elpa_hh_plan& p) {
  return p.path >= ELPA_PATH_AUTO && p.path <= ELPA_PATH_WY && p.k >= 0 && p.steps >= 0 &&
         p.order >= ELPA_ORDER_AUTO && p.order <= ELPA_ORDER_XCD && p.streams >= 0 &&
         p.streams <= 8 && p.batch >= ELPA_BATCH_AUTO && p.batch <= ELPA_BATCH_DIAGONAL;
}

}  // namespace

bool tuner_lookup(int32_t dtype, int64_t nbw, int64_t n, int64_t nev, elpa_hh_plan* out) {
  Cache& c = Cache::get();
  std::lock_guard<std::mutex> g(c.mu);
  const auto it = c.plans.find(key_of(dtype, nbw, n, nev));
  if (it == c.plans.end()) return false;
  *out = it->second;
  return true;
}

}  // namespace ehh

extern "C" {

int elpa_hh_tuner_set(int32_t dtype, int64_t nbw, int64_t n, int64_t nev,
                      const elpa_hh_plan* plan) {
  if (!plan || nbw < 1 || n < 0 || nev < 0 || !ehh::plan_valid(*plan)) return ELPA_ERR_ARG;
  if (!elpa_hh_plan_supported(nbw, dtype, plan)) return ELPA_ERR_PLAN;
  ehh::Cache& c = ehh::Cache::get();
  std::lock_guard<std::mutex> g(c.mu);
  c.plans[ehh::key_of(dtype, nbw, n, nev)] = *plan;
  return ELPA_OK;
}

int elpa_hh_tuner_get(int32_t dtype, int64_t nbw, int64_t n, int64_t nev, elpa_hh_plan* out) {
  if (!out) return ELPA_ERR_ARG;
  return ehh::tuner_lookup(dtype, nbw, n, nev, out) ? 1 : 0;
}

int64_t elpa_hh_tuner_size(void) {
  ehh::Cache& c = ehh::Cache::get();
  std::lock_guard<std::mutex> g(c.mu);
  return (int64_t)c.plans.size();
}

void elpa_hh_tuner_clear(void) {
  ehh::Cache& c = ehh::Cache::get();
  std::lock_guard<std::mutex> g(c.mu);
  c.plans.clear();
}

int elpa_hh_tuner_save(const char* path) {
  if (!path) return ELPA_ERR_ARG;
  ehh::Cache& c = ehh::Cache::get();
  std::lock_guard<std::mutex> g(c.mu);
  FILE* f = std::fopen(path, "w");
  if (!f) return ELPA_ERR_ARG;
  std::fprintf(f, "elpa_hh_tuner 1\n");
  std::fprintf(f, "# dtype nbw n_class nev_class path k steps order streams\n");
  for (const auto& kv : c.plans) {
    const elpa_hh_plan& p = kv.second;
    std::fprintf(f, "%d %lld %lld %lld %d %d %d %d %d\n", (int)std::get<0>(kv.first),
                 (long long)std::get<1>(kv.first), (long long)std::get<2>(kv.first),
                 (long long)std::get<3>(kv.first), p.path, p.k, p.steps, p.order, p.streams);
  }
  const bool ok = std::fclose(f) == 0;
  return ok ? ELPA_OK : ELPA_ERR_ARG;
}

int elpa_hh_tuner_load(const char* path) {
  if (!path) return ELPA_ERR_ARG;
  FILE* f = std::fopen(path, "r");
  if (!f) return ELPA_ERR_ARG;
  char line[512];
  std::map<ehh::Key, elpa_hh_plan> got;
  bool ok = std::fgets(line, sizeof line, f) && std::strncmp(line, "elpa_hh_tuner 1", 15) == 0;
  while (ok && std::fgets(line, sizeof line, f)) {
    if (line[0] == '#' || line[0] == '\n') continue;
    int dt, path_, k, steps, order, streams;
    long long nbw, nc, ec;
    if (std::sscanf(line, "%d %lld %lld %lld %d %d %d %d %d", &dt, &nbw, &nc, &ec, &path_, &k,
                    &steps, &order, &streams) != 9) {
      ok = false;
      break;
    }
    const elpa_hh_plan p{path_, k, steps, order, streams, 0};
    if (nbw < 1 || nc < 0 || ec < 0 || !ehh::plan_valid(p) ||
        !elpa_hh_plan_supported(nbw, dt, &p)) {
      ok = false;
      break;
    }
    got[ehh::Key{dt, (int64_t)nbw, (int64_t)nc, (int64_t)ec}] = p;
  }
  std::fclose(f);
  if (!ok) return ELPA_ERR_ARG;
  ehh::Cache& c = ehh::Cache::get();
  std::lock_guard<std::mutex> g(c.mu);
  for (const auto& kv : got) c.plans[kv.first] = kv.second;
  return ELPA_OK;
}

int elpa_hh_tune(int64_t n, int64_t nev, int64_t nbw, const void* hh, const void* tau,
                 const void* Q, int64_t ldq, int32_t dtype, void* stream, int32_t level,
                 elpa_hh_plan* best) {
  if (level < 0 || level > 2) return ELPA_ERR_ARG;
  if (n <= 1 || nev <= 0 || nbw < 1 || ldq < n || !hh || !tau || !Q) return ELPA_ERR_ARG;
  if (dtype != ELPA_R64 && dtype != ELPA_R32 && dtype != ELPA_C64) return ELPA_ERR_DTYPE;
  const int64_t es = dtype == ELPA_C64 ? 16 : (dtype == ELPA_R32 ? 4 : 8);
  // candidates: level 0 each kernel family's default k, level 1 every compiled
  // k, level 2 also explicit tile heights; each with 1 and 2 stripe groups
  std::vector<elpa_hh_plan> cand;
  const int steps_list[] = {0, 2, 4, 8, 16};
  const int nsteps = level == 2 ? 5 : 1;
  for (int fam : {ELPA_PATH_SPLIT, ELPA_PATH_WY, ELPA_PATH_STRIPE}) {
    std::vector<int> ks;
    if (level == 0) {
      const elpa_hh_plan def{fam, 0, 0, 0, 0, 0};
      if (elpa_hh_plan_supported(nbw, dtype, &def)) ks.push_back(0);
    } else {
      int cnt = 0;
      const ehh::StripeEntry* tab = fam == ELPA_PATH_SPLIT ? ehh::split_table(&cnt)
                                    : fam == ELPA_PATH_WY  ? ehh::wy_table(&cnt)
                                                           : ehh::stripe_table(&cnt);
      for (int i = 0; i < cnt; ++i)
        if (tab[i].dtype == dtype && tab[i].nb == nbw) ks.push_back(tab[i].k);
    }
    for (int k : ks)
      for (int si = 0; si < nsteps; ++si)
        for (int streams : {1, 2}) cand.push_back(elpa_hh_plan{fam, k, steps_list[si], 0, streams, 0});
  }
  if (cand.empty()) cand.push_back(elpa_hh_plan{ELPA_PATH_REF, 0, 0, 0, 0, 0});
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  void* scratch = nullptr;
  // the caller's Q spans ldq*(nev-1) + n elements
  const size_t bytes = ((size_t)ldq * (size_t)(nev - 1) + (size_t)n) * (size_t)es;
  if (hipMallocAsync(&scratch, bytes, st) != hipSuccess) return ELPA_ERR_NOMEM;
  hipEvent_t a = nullptr, b = nullptr;
  bool ok = hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess &&
            hipMemcpyAsync(scratch, Q, bytes, hipMemcpyDeviceToDevice, st) == hipSuccess;
  float best_ms = -1.f;
  elpa_hh_plan win{};
  const int reps = 2;
  int rc = ELPA_OK;
  for (size_t i = 0; ok && i < cand.size(); ++i) {
    const elpa_hh_plan& p = cand[i];
    // warm-up (also the first use of the kernel, and the argument checks)
    rc = elpa_hh_trafo_plan(n, nev, nbw, hh, tau, scratch, ldq, dtype, stream, &p);
    if (rc != ELPA_OK) {
      ok = false;
      break;
    }
    ok = hipEventRecord(a, st) == hipSuccess;
    for (int r = 0; ok && r < reps; ++r)
      ok = elpa_hh_trafo_plan(n, nev, nbw, hh, tau, scratch, ldq, dtype, stream, &p) == ELPA_OK;
    ok = ok && hipEventRecord(b, st) == hipSuccess && hipEventSynchronize(b) == hipSuccess;
    float ms = 0.f;
    ok = ok && hipEventElapsedTime(&ms, a, b) == hipSuccess;
    if (ok && (best_ms < 0.f || ms < best_ms)) {
      best_ms = ms;
      win = p;
    }
  }
  (void)hipFreeAsync(scratch, st);
  (void)hipStreamSynchronize(st);
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  if (rc != ELPA_OK) return rc;
  if (!ok || best_ms < 0.f) return ELPA_ERR_DEVICE;
  {
    ehh::Cache& c = ehh::Cache::get();
    std::lock_guard<std::mutex> g(c.mu);
    c.plans[ehh::key_of(dtype, nbw, n, nev)] = win;
  }
  if (best) *best = win;
  return ELPA_OK;
}

int elpa_hh_tune_batched(const elpa_hh_problem* probs, int64_t count, void* stream, int32_t level,
                         elpa_hh_plan* best) {
  if (level < 0 || level > 2 || count <= 0 || !probs) return ELPA_ERR_ARG;
  // scratch copies of every Q (the span ldq*(nev-1)+n of each), 256-aligned
  std::vector<elpa_hh_problem> work(probs, probs + count);
  std::vector<size_t> off(count, 0), len(count, 0);
  size_t total = 0;
  for (int64_t i = 0; i < count; ++i) {
    const elpa_hh_problem& p = probs[i];
    const int64_t es = p.dtype == ELPA_C64 ? 16 : p.dtype == ELPA_R64 ? 8 : p.dtype == ELPA_R32 ? 4 : 0;
    if (es == 0) return ELPA_ERR_DTYPE;
    if (p.n < 0 || p.nev < 0 || p.nbw < 1) return ELPA_ERR_ARG;
    if (p.n <= 1 || p.nev == 0) continue;
    if (p.ldq < p.n || !p.Q) return ELPA_ERR_ARG;
    if (p.nev > 1 && p.ldq > (INT64_MAX / es - p.n) / (p.nev - 1)) return ELPA_ERR_ARG;
    len[i] = ((size_t)p.ldq * (size_t)(p.nev - 1) + (size_t)p.n) * (size_t)es;
    off[i] = total;
    total += (len[i] + 255) / 256 * 256;
  }
  // candidates: uniform plans that every problem of the batch can run
  std::vector<elpa_hh_plan> cand;
  const int steps_list[] = {0, 2, 4, 8, 16};
  const int nsteps = level == 2 ? 5 : 1;
  for (int fam : {ELPA_PATH_SPLIT, ELPA_PATH_WY, ELPA_PATH_STRIPE}) {
    std::set<int> ks;
    if (level == 0) {
      ks.insert(0);
    } else {
      int cnt = 0;
      const ehh::StripeEntry* tab = fam == ELPA_PATH_SPLIT ? ehh::split_table(&cnt)
                                    : fam == ELPA_PATH_WY  ? ehh::wy_table(&cnt)
                                                           : ehh::stripe_table(&cnt);
      for (int i = 0; i < cnt; ++i) ks.insert(tab[i].k);
    }
    for (int k : ks) {
      if (fam == ELPA_PATH_SPLIT) {
        // the two-lane family's batched schedules: one launch, or the
        // diagonal sequence at each tile height (one stream either way)
        const elpa_hh_plan one{fam, k, 0, 0, 1, ELPA_BATCH_ONE_LAUNCH};
        if (elpa_hh_workspace_bytes_batched(probs, count, &one) >= 0) cand.push_back(one);
        for (int si = 0; si < nsteps; ++si) {
          const elpa_hh_plan p{fam, k, steps_list[si], 0, 1, ELPA_BATCH_DIAGONAL};
          if (elpa_hh_workspace_bytes_batched(probs, count, &p) >= 0) cand.push_back(p);
        }
        continue;
      }
      for (int si = 0; si < nsteps; ++si)
        for (int streams : {1, 2}) {
          const elpa_hh_plan p{fam, k, steps_list[si], 0, streams, 0};
          if (elpa_hh_workspace_bytes_batched(probs, count, &p) >= 0) cand.push_back(p);
        }
    }
  }
  if (cand.empty()) cand.push_back(elpa_hh_plan{ELPA_PATH_REF, 0, 0, 0, 0, 0});
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char* scratch = nullptr;
  if (total > 0 && hipMallocAsync((void**)&scratch, total, st) != hipSuccess) return ELPA_ERR_NOMEM;
  bool ok = true;
  for (int64_t i = 0; ok && i < count; ++i) {
    if (len[i] == 0) continue;
    work[i].Q = scratch + off[i];
    ok = hipMemcpyAsync(work[i].Q, probs[i].Q, len[i], hipMemcpyDeviceToDevice, st) == hipSuccess;
  }
  hipEvent_t a = nullptr, b = nullptr;
  ok = ok && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess;
  float best_ms = -1.f;
  elpa_hh_plan win{};
  const int reps = 2;
  int rc = ELPA_OK;
  for (size_t c = 0; ok && c < cand.size(); ++c) {
    const elpa_hh_plan& p = cand[c];
    rc = elpa_hh_trafo_batched(work.data(), count, stream, &p);  // warm-up and checks
    if (rc != ELPA_OK) {
      ok = false;
      break;
    }
    ok = hipEventRecord(a, st) == hipSuccess;
    for (int r = 0; ok && r < reps; ++r)
      ok = elpa_hh_trafo_batched(work.data(), count, stream, &p) == ELPA_OK;
    ok = ok && hipEventRecord(b, st) == hipSuccess && hipEventSynchronize(b) == hipSuccess;
    float ms = 0.f;
    ok = ok && hipEventElapsedTime(&ms, a, b) == hipSuccess;
    if (ok && (best_ms < 0.f || ms < best_ms)) {
      best_ms = ms;
      win = p;
    }
  }
  if (scratch) (void)hipFreeAsync(scratch, st);
  (void)hipStreamSynchronize(st);
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  if (rc != ELPA_OK) return rc;
  if (!ok || best_ms < 0.f) return ELPA_ERR_DEVICE;
  if (best) *best = win;
  return ELPA_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// On-the-fly autotuning over a sequence of solves (C ABI in include/elpa_hh.h)
// ---------------------------------------------------------------------------
struct elpa_hh_autotune_state {
  int32_t level = 0, dtype = 0;
  int64_t n = 0, nev = 0, nbw = 0;
  std::vector<elpa_hh_plan> cand;
  std::vector<double> ms;  // -1: not timed
  int64_t next = -1;       // -1: warm-up step pending
  int64_t pending = -1;    // candidate whose events are not read yet
  hipEvent_t a = nullptr, b = nullptr;
};

namespace ehh {
namespace {

std::vector<elpa_hh_plan> autotune_candidates(int32_t level, int64_t nbw, int32_t dtype,
                                              const elpa_hh_plan* fixed) {
  std::vector<elpa_hh_plan> out;
  const elpa_hh_plan fx = fixed ? *fixed : elpa_hh_plan{0, 0, 0, 0, 0, 0};
  const int steps_all[] = {0, 2, 4, 8, 16};
  for (int fam : {ELPA_PATH_SPLIT, ELPA_PATH_WY, ELPA_PATH_STRIPE}) {
    if (fx.path && fx.path != fam) continue;
    std::vector<int> ks;
    if (fx.k) {
      ks.push_back(fx.k);
    } else if (level == ELPA_AUTOTUNE_FAST) {
      ks.push_back(0);
    } else {
      int cnt = 0;
      const StripeEntry* tab = fam == ELPA_PATH_SPLIT ? split_table(&cnt)
                               : fam == ELPA_PATH_WY  ? wy_table(&cnt)
                                                      : stripe_table(&cnt);
      for (int i = 0; i < cnt; ++i)
        if (tab[i].dtype == dtype && tab[i].nb == nbw) ks.push_back(tab[i].k);
    }
    std::vector<int> steps, streams;
    if (fx.steps)
      steps.push_back(fx.steps);
    else if (level == ELPA_AUTOTUNE_FAST)
      steps.push_back(0);
    else
      steps.assign(std::begin(steps_all), std::end(steps_all));
    if (fx.streams)
      streams.push_back(fx.streams);
    else if (level == ELPA_AUTOTUNE_FAST)
      streams.push_back(0);
    else
      streams = {1, 2};
    for (int k : ks)
      for (int s : steps)
        for (int ns : streams) {
          const elpa_hh_plan p{fam, k, s, fx.order, ns, 0};
          if (elpa_hh_plan_supported(nbw, dtype, &p)) out.push_back(p);
        }
  }
  return out;
}

// read the pending timing (waits for the step's end event)
int autotune_settle(elpa_hh_autotune_state* st) {
  if (st->pending < 0) return ELPA_OK;
  float ms = 0.f;
  if (hipEventSynchronize(st->b) != hipSuccess ||
      hipEventElapsedTime(&ms, st->a, st->b) != hipSuccess)
    return ELPA_ERR_DEVICE;
  st->ms[(size_t)st->pending] = ms;
  st->pending = -1;
  return ELPA_OK;
}

int64_t autotune_best_index(const elpa_hh_autotune_state* st) {
  int64_t best = -1;
  for (size_t i = 0; i < st->ms.size(); ++i)
    if (st->ms[i] >= 0.0 && (best < 0 || st->ms[i] < st->ms[(size_t)best])) best = (int64_t)i;
  return best;
}

bool autotune_events(elpa_hh_autotune_state* st) {
  return hipEventCreate(&st->a) == hipSuccess && hipEventCreate(&st->b) == hipSuccess;
}

}  // namespace
}  // namespace ehh

extern "C" {

elpa_hh_autotune_state* elpa_hh_autotune_setup(int32_t level, int64_t n, int64_t nev,
                                               int64_t nbw, int32_t dtype,
                                               const elpa_hh_plan* fixed) {
  if (level != ELPA_AUTOTUNE_FAST && level != ELPA_AUTOTUNE_MEDIUM) return nullptr;
  if (n <= 1 || nev <= 0 || nbw < 1) return nullptr;
  if (dtype != ELPA_R64 && dtype != ELPA_R32 && dtype != ELPA_C64) return nullptr;
  if (fixed && (fixed->k < 0 || fixed->steps < 0 || fixed->streams < 0 || fixed->streams > 8 ||
                fixed->batch < ELPA_BATCH_AUTO || fixed->batch > ELPA_BATCH_DIAGONAL))
    return nullptr;
  auto* st = new elpa_hh_autotune_state();
  st->level = level;
  st->dtype = dtype;
  st->n = n;
  st->nev = nev;
  st->nbw = nbw;
  st->cand = ehh::autotune_candidates(level, nbw, dtype, fixed);
  st->ms.assign(st->cand.size(), -1.0);
  if (st->cand.empty()) {
    elpa_hh_autotune_free(st);
    return nullptr;
  }
  return st;
}

int64_t elpa_hh_autotune_candidates(const elpa_hh_autotune_state* st) {
  return st ? (int64_t)st->cand.size() : -1;
}

int elpa_hh_autotune_step(elpa_hh_autotune_state* st, const void* hh, const void* tau, void* Q,
                          int64_t ldq, void* stream, int32_t* tuning) {
  if (!st || !tuning) return ELPA_ERR_ARG;
  // the events belong to the device current at the first step
  if (!st->a && !ehh::autotune_events(st)) return ELPA_ERR_DEVICE;
  int rc = ehh::autotune_settle(st);
  if (rc != ELPA_OK) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (st->next < 0) {  // warm-up: the first candidate, untimed
    rc = elpa_hh_trafo_plan(st->n, st->nev, st->nbw, hh, tau, Q, ldq, st->dtype, stream,
                            &st->cand[0]);
    if (rc == ELPA_OK) st->next = 0;
    *tuning = 1;
    return rc;
  }
  if (st->next < (int64_t)st->cand.size()) {
    const int64_t i = st->next;
    if (hipEventRecord(st->a, s) != hipSuccess) return ELPA_ERR_DEVICE;
    rc = elpa_hh_trafo_plan(st->n, st->nev, st->nbw, hh, tau, Q, ldq, st->dtype, stream,
                            &st->cand[(size_t)i]);
    if (rc != ELPA_OK) return rc;
    if (hipEventRecord(st->b, s) != hipSuccess) return ELPA_ERR_DEVICE;
    st->pending = i;
    st->next = i + 1;
    *tuning = st->next < (int64_t)st->cand.size() ? 1 : 0;
    return ELPA_OK;
  }
  *tuning = 0;
  const int64_t b = ehh::autotune_best_index(st);
  return elpa_hh_trafo_plan(st->n, st->nev, st->nbw, hh, tau, Q, ldq, st->dtype, stream,
                            &st->cand[(size_t)(b < 0 ? 0 : b)]);
}

int elpa_hh_autotune_best(elpa_hh_autotune_state* st, elpa_hh_plan* best) {
  if (!st || !best) return ELPA_ERR_ARG;
  const int rc = ehh::autotune_settle(st);
  if (rc != ELPA_OK) return rc;
  const int64_t b = ehh::autotune_best_index(st);
  if (b < 0) return ELPA_ERR_ARG;
  *best = st->cand[(size_t)b];
  return ELPA_OK;
}

int elpa_hh_autotune_set_best(elpa_hh_autotune_state* st) {
  elpa_hh_plan best{};
  const int rc = elpa_hh_autotune_best(st, &best);
  if (rc != ELPA_OK) return rc;
  return elpa_hh_tuner_set(st->dtype, st->nbw, st->n, st->nev, &best);
}

int elpa_hh_autotune_save(elpa_hh_autotune_state* st, const char* path) {
  if (!st || !path) return ELPA_ERR_ARG;
  const int rc = ehh::autotune_settle(st);
  if (rc != ELPA_OK) return rc;
  FILE* f = std::fopen(path, "w");
  if (!f) return ELPA_ERR_ARG;
  std::fprintf(f, "elpa_hh_autotune 1\n");
  std::fprintf(f, "%d %d %lld %lld %lld %lld %lld\n", st->level, st->dtype, (long long)st->n,
               (long long)st->nev, (long long)st->nbw, (long long)st->next,
               (long long)st->cand.size());
  for (size_t i = 0; i < st->cand.size(); ++i) {
    const elpa_hh_plan& p = st->cand[i];
    std::fprintf(f, "%d %d %d %d %d %.6f\n", p.path, p.k, p.steps, p.order, p.streams,
                 st->ms[i]);
  }
  return std::fclose(f) == 0 ? ELPA_OK : ELPA_ERR_ARG;
}

elpa_hh_autotune_state* elpa_hh_autotune_load(const char* path) {
  if (!path) return nullptr;
  FILE* f = std::fopen(path, "r");
  if (!f) return nullptr;
  char line[512];
  auto* st = new elpa_hh_autotune_state();
  long long n = 0, nev = 0, nbw = 0, next = 0, cnt = 0;
  bool ok = std::fgets(line, sizeof line, f) && std::strncmp(line, "elpa_hh_autotune 1", 18) == 0;
  ok = ok && std::fgets(line, sizeof line, f) &&
       std::sscanf(line, "%d %d %lld %lld %lld %lld %lld", &st->level, &st->dtype, &n, &nev, &nbw,
                   &next, &cnt) == 7;
  ok = ok && n > 1 && nev > 0 && nbw > 0 && cnt > 0 && cnt < 100000 && next >= -1 && next <= cnt;
  for (long long i = 0; ok && i < cnt; ++i) {
    elpa_hh_plan p{};
    double ms = -1.0;
    ok = std::fgets(line, sizeof line, f) &&
         std::sscanf(line, "%d %d %d %d %d %lf", &p.path, &p.k, &p.steps, &p.order, &p.streams,
                     &ms) == 6 &&
         elpa_hh_plan_supported(nbw, st->dtype, &p);
    st->cand.push_back(p);
    st->ms.push_back(ms);
  }
  std::fclose(f);
  st->n = n;
  st->nev = nev;
  st->nbw = nbw;
  st->next = next;
  if (!ok) {
    elpa_hh_autotune_free(st);
    return nullptr;
  }
  return st;
}

void elpa_hh_autotune_free(elpa_hh_autotune_state* st) {
  if (!st) return;
  if (st->pending >= 0 && st->b) (void)hipEventSynchronize(st->b);
  if (st->a) (void)hipEventDestroy(st->a);
  if (st->b) (void)hipEventDestroy(st->b);
  delete st;
}

}  // extern "C"
