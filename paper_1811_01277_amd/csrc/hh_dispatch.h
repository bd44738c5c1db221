// Launcher tables shared between the kernel translation unit and the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/elpa_hh.h"

namespace ehh {

// Tiling of the diagonal launch schedule: steps = chase steps per tile
// (0 = library choice); xcd = number of consecutive-tile groups the workgroup
// ids are dealt to round robin (1 = linear order, 8 = one group per XCD);
// streams = stripe groups run as separate launch sequences on concurrent
// streams (1 = the caller's stream only).
struct TileOpts {
  int64_t steps;
  int xcd;
  int streams;
  int batch;  // ELPA_BATCH_* (batched calls of the two-lane kernel)
  int order;  // ELPA_ORDER_* as given (the one-launch batched schedule groups
              // each problem's stripes on one die unless ELPA_ORDER_LINEAR)
};

using StripeLaunch = hipError_t (*)(const void* hh, const void* tau, void* Q, int64_t ldq,
                                    int64_t n, int64_t nev, TileOpts opt, hipStream_t st,
                                    int num_cu);
using BatchedLaunch = hipError_t (*)(const elpa_hh_problem* probs, const int64_t* idx,
                                     int64_t cnt, TileOpts opt, hipStream_t st, int num_cu);
// Device workspace one problem's call allocates (bytes).
using WorkspaceFn = size_t (*)(int64_t n, int64_t nev);
// A prepared batched group (elpa_hh_batch_create): device workspace and
// tables owned for the object's lifetime; run() only launches kernels.
class PreparedGroup {
 public:
  virtual ~PreparedGroup() = default;
  virtual hipError_t run(hipStream_t st) = 0;
  virtual size_t bytes() const = 0;  // device bytes owned
};
using PrepareFn = hipError_t (*)(const elpa_hh_problem* probs, const int64_t* idx, int64_t cnt,
                                 TileOpts opt, int num_cu, PreparedGroup** out);

// Same as StripeLaunch on a caller-provided device workspace of at least
// WorkspaceFn(n, nev) bytes (nothing allocated or freed).
using StripeLaunchWs = hipError_t (*)(const void* hh, const void* tau, void* Q, int64_t ldq,
                                      int64_t n, int64_t nev, TileOpts opt, hipStream_t st,
                                      int num_cu, void* ws);
using RefLaunch = hipError_t (*)(const void* hh, const void* tau, void* Q, int64_t ldq,
                                 int64_t n, int64_t nev, int64_t nb, hipStream_t st);

struct StripeEntry {
  int path;   // ELPA_PATH_STRIPE, ELPA_PATH_SPLIT or ELPA_PATH_WY
  int dtype;
  int nb;
  int k;
  int occ;  // waves per SIMD the kernel is compiled for
  StripeLaunch fn;
  BatchedLaunch batched;  // null: no batched form
  WorkspaceFn workspace;
  StripeLaunchWs with_ws;  // null: the family has no caller-workspace form
  PrepareFn prepare;       // null: the family has no prepared batched form
};

const StripeEntry* stripe_table(int* size);  // one lane per column
const StripeEntry* split_table(int* size);   // two lanes per column, packed reflectors
const StripeEntry* wy_table(int* size);      // compact-WY sub-groups on MFMA
RefLaunch ref_launcher(int dtype);

// Device address and size of the current device's fixed scratch (the
// allocation-free entry point's workspace; hh_noalloc.hip).
hipError_t noalloc_scratch(void** out, size_t* bytes);

// Tuned plan of the size class of (n, nev), if the tuner holds one.
bool tuner_lookup(int32_t dtype, int64_t nbw, int64_t n, int64_t nev, elpa_hh_plan* out);

// Timing of the main kernel sequence (the tile launches of the stripe paths,
// the single launch of the reference path) of the latest call made on the
// calling host thread, while enabled with elpa_hh_profile_enable: an event
// pair around the whole sequence on the caller's stream, and one around every
// launch on the stream it is launched on.
struct ProfState {
  bool on = false;
  int dev = -1;
  hipEvent_t a = nullptr, b = nullptr;
  std::vector<hipEvent_t> ev;  // per launch: before, after
  bool started = false, recorded = false;
  int64_t launches = 0;
  int path = 0, k = 0, streams = 1;
  int64_t steps = 0;
};
ProfState& prof_state();  // thread-local

// Brackets one launch sequence on `st`: an event before the first sequence of
// a call, an event after every sequence (the last one counts), and before() /
// after() around each launch.
class ProfScope {
 public:
  ProfScope(hipStream_t st, int k, int64_t steps, int streams = 1) : st_(st) {
    ProfState& p = prof_state();
    int dev = -1;
    on_ = p.on && p.a && (hipGetDevice(&dev) == hipSuccess) && dev == p.dev;
    if (!on_) return;
    if (!p.started && hipEventRecord(p.a, st) == hipSuccess) p.started = true;
    p.k = k;
    p.steps = steps;
    p.streams = streams;
  }
  void before(hipStream_t s) {
    if (!on_) return;
    ProfState& p = prof_state();
    const size_t i = 2 * (size_t)p.launches;
    while (p.ev.size() < i + 2) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) {
        on_ = false;
        return;
      }
      p.ev.push_back(e);
    }
    (void)hipEventRecord(p.ev[i], s);
  }
  void after(hipStream_t s) {
    if (!on_) return;
    ProfState& p = prof_state();
    (void)hipEventRecord(p.ev[2 * (size_t)p.launches + 1], s);
    ++p.launches;
  }
  void end() {
    if (!on_) return;
    ProfState& p = prof_state();
    if (hipEventRecord(p.b, st_) == hipSuccess) p.recorded = p.started;
    on_ = false;
  }
  ~ProfScope() { end(); }

 private:
  hipStream_t st_;
  bool on_ = false;
};

}  // namespace ehh
