// Scheduling and staging helpers shared by the stripe kernel families of the
// tridiagonal->band back-transformation: the diagonal launch schedule over
// (stripe, sweep block, group of chase steps) tiles, the batched problem
// descriptors, stream-ordered upload of small host tables, and compile-time
// loops used by the fully unrolled step bodies.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <vector>

#include "hh_common.h"

namespace ehh {

// Geometry of one problem of the stripe path (device copy used by the
// batched kernels).
struct ProblemDesc {
  const void* hh;
  const void* tau;
  void* Q;
  void* Qs;
  int64_t n, nev, ldq, rows_pad;
  int G, M, S;
  int tile0;   // first 64x64 conversion tile of this problem (rows_pad/64 * GT tiles)
  int otile0;  // first conversion tile back (ceil(n/64) * GT tiles)
  int GT;      // 64-column conversion tiles per row band, ceil(nev/64)
  int ptile0;     // first reflector-packing group of this problem (split path)
  const void* P;  // packed reflectors (split path), else null
  int64_t Jmax;   // chase steps of the longest sweep, ceil((n-1)/nbw)
  int unit0;      // first workgroup of this problem in a one-launch batched call
  int pad_;
  const void* Bt;  // first packed step record of each sweep block (split path)
};

// One launch's share of one problem in the batched diagonal schedule:
// blocks [m0, m0 + mcount) of problem p, every stripe; tiles [tile0,
// tile0 + mcount*G) of the launch.
struct DiagEntry {
  int p;
  int m0;
  int mcount;
  int tile0;
};

// Tile index of workgroup b of a launch of U workgroups.  Workgroup ids are
// dealt to the accelerator dies round robin (b -> die b % xcd); giving each
// die a contiguous run of tile indices keeps tiles of one sweep block, which
// read the same reflectors, on one die's L2.  xcd <= 1: identity.
__device__ __forceinline__ int tile_of(int b, int U, int xcd) {
  if (xcd <= 1) return b;
  const int x = b % xcd, i = b / xcd;
  const int per = U / xcd, rem = U % xcd;
  return x * per + (x < rem ? x : rem) + i;
}

// index i with key(d[i]) <= key < key(d[i+1]) (d sorted by key)
template <typename T, int T::*F>
__device__ __forceinline__ int find_by(const T* __restrict__ d, int count, int key) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d[mid].*F <= key)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Compile-time loop o = N-1, N-2, ..., 0 (every body gets a constant o, so
// the window indices stay static without relying on the unroller's budget).
template <int N>
struct RevFor {
  template <typename F>
  static __device__ __forceinline__ void run(F&& f) {
    f(std::integral_constant<int, N - 1>{});
    RevFor<N - 1>::run(f);
  }
};
template <>
struct RevFor<0> {
  template <typename F>
  static __device__ __forceinline__ void run(F&&) {}
};

// Compile-time loop i = 0, 1, ..., N-1.
template <int N, int I = 0>
struct FwdFor {
  template <typename F>
  static __device__ __forceinline__ void run(F&& f) {
    if constexpr (I < N) {
      f(std::integral_constant<int, I>{});
      FwdFor<N, I + 1>::run(f);
    }
  }
};

// An SGPR zero that the compiler cannot compute before the VGPR value d is
// available: adding it to an address keeps the load after the instruction
// that produced d instead of letting the scheduler hoist it.
__device__ __forceinline__ int zero_after(double d) {
  int z;
  asm("s_mov_b32 %0, 0" : "=s"(z) : "v"(d));
  return z;
}
__device__ __forceinline__ int zero_after(float d) {
  int z;
  asm("s_mov_b32 %0, 0" : "=s"(z) : "v"(d));
  return z;
}
__device__ __forceinline__ int zero_after(z64 d) { return zero_after(d.re); }

inline size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Workspace of one call on the current device, valid in the order of `st`:
// a block of the library's workspace cache (hh_ws.cpp) that no pending work
// uses, or, while `st` is being captured into a graph, a stream-ordered
// allocation that the graph owns.  A request above the device's total memory
// fails at once with hipErrorOutOfMemory; a failed allocation leaves no error
// behind for the next runtime call to report.
hipError_t ws_alloc(void** p, size_t bytes, hipStream_t st);
// Returns a ws_alloc block after the work enqueued on `st` so far: the cache
// hands it out again to later work on `st` at once, and to work on other
// streams once that work has completed.
hipError_t ws_free(void* p, hipStream_t st);

// Stream-ordered host->device upload of small host tables.  hipMemcpyAsync
// from pageable memory copies at call time, but a destination obtained from
// hipMallocAsync is only valid in stream order (earlier work on the stream may
// still use the recycled memory), so tables are staged in pinned host buffers
// and copied asynchronously; a buffer is reused only after the event recorded
// behind its copy has completed.  One pool per device.
class PinnedStaging {
 public:
  static PinnedStaging& for_device(int dev) {
    static std::mutex mu;
    static std::vector<PinnedStaging*> pools;
    std::lock_guard<std::mutex> g(mu);
    if (dev < 0) dev = 0;
    if ((size_t)dev >= pools.size()) pools.resize((size_t)dev + 1, nullptr);
    if (!pools[(size_t)dev]) pools[(size_t)dev] = new PinnedStaging();
    return *pools[(size_t)dev];
  }

  // copy `bytes` from host `src` to device `dst` in stream order on `st`
  hipError_t upload(void* dst, const void* src, size_t bytes, hipStream_t st) {
    if (bytes == 0) return hipSuccess;
    std::lock_guard<std::mutex> g(mu_);
    Buf* b = nullptr;
    for (Buf& x : bufs_) {
      if (x.cap >= bytes && hipEventQuery(x.ev) == hipSuccess) {
        b = &x;
        break;
      }
    }
    if (!b) {
      Buf nb{};
      nb.cap = std::max<size_t>(bytes, 1 << 16);
      hipError_t e = hipHostMalloc(&nb.p, nb.cap, hipHostMallocDefault);
      if (e != hipSuccess) return e;
      e = hipEventCreateWithFlags(&nb.ev, hipEventDisableTiming);
      if (e != hipSuccess) {
        (void)hipHostFree(nb.p);
        return e;
      }
      bufs_.push_back(nb);
      b = &bufs_.back();
    }
    std::memcpy(b->p, src, bytes);
    hipError_t e = hipMemcpyAsync(dst, b->p, bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    return hipEventRecord(b->ev, st);
  }

 private:
  struct Buf {
    void* p;
    size_t cap;
    hipEvent_t ev;
  };
  std::mutex mu_;
  std::vector<Buf> bufs_;
};

// Fork/join of a launch sequence over internal streams.  With ns == 1 the
// caller's stream is used directly.  Otherwise ns library streams (created
// once, default priority, non-blocking) wait for an event recorded on the
// caller's stream, and join() makes the caller's stream wait for events
// recorded behind the work enqueued on them.  Each (device, caller stream)
// pair has a pool of its own, so calls on different caller streams fork onto
// different library streams and run concurrently; a pool is locked from fork
// to join so that concurrent callers on the same stream do not interleave
// their fork/join events.  Past kMaxPools caller streams on a device, the
// further ones share one overflow pool.
class StreamFork {
 public:
  static constexpr int kMax = 8;

  StreamFork(hipStream_t caller, int ns) : caller_(caller), ns_(ns < 1 ? 1 : (ns > kMax ? kMax : ns)) {
    streams_[0] = caller;
    if (ns_ == 1) return;
    int dev = 0;
    err_ = hipGetDevice(&dev);
    if (err_ != hipSuccess) return;
    pool_ = &Pool::for_stream(dev, caller);
    lock_ = std::unique_lock<std::mutex>(pool_->mu);
    err_ = pool_->ensure(ns_);
    if (err_ != hipSuccess) return;
    err_ = hipEventRecord(pool_->fork, caller);
    for (int i = 0; i < ns_ && err_ == hipSuccess; ++i) {
      streams_[i] = pool_->s[(size_t)i];
      err_ = hipStreamWaitEvent(streams_[i], pool_->fork, 0);
    }
  }
  ~StreamFork() { (void)join(); }
  hipError_t error() const { return err_; }
  int count() const { return ns_; }
  hipStream_t stream(int i) const { return streams_[i]; }

  hipError_t join() {
    if (ns_ == 1 || joined_ || !pool_) return err_;
    joined_ = true;
    for (int i = 0; i < ns_; ++i) {
      hipError_t e = hipEventRecord(pool_->join[(size_t)i], streams_[i]);
      if (e == hipSuccess) e = hipStreamWaitEvent(caller_, pool_->join[(size_t)i], 0);
      if (e != hipSuccess && err_ == hipSuccess) err_ = e;
    }
    lock_ = std::unique_lock<std::mutex>();
    return err_;
  }

 private:
  struct Pool {
    std::mutex mu;
    std::vector<hipStream_t> s;
    std::vector<hipEvent_t> join;
    hipEvent_t fork = nullptr;
    hipError_t ensure(int n) {
      if (!fork) {
        const hipError_t e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
        if (e != hipSuccess) return e;
      }
      while ((int)s.size() < n) {
        hipStream_t x = nullptr;
        hipEvent_t ev = nullptr;
        hipError_t e = hipStreamCreateWithFlags(&x, hipStreamNonBlocking);
        if (e != hipSuccess) return e;
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) return e;
        s.push_back(x);
        join.push_back(ev);
      }
      return hipSuccess;
    }
    static Pool& for_stream(int dev, hipStream_t caller) {
      struct Entry {
        int dev;
        hipStream_t caller;
        Pool* pool;
      };
      static std::mutex mu;
      static std::vector<Entry> pools;
      std::lock_guard<std::mutex> g(mu);
      for (const Entry& e : pools)
        if (e.dev == dev && e.caller == caller) return *e.pool;
      int on_dev = 0;
      for (const Entry& e : pools) on_dev += e.dev == dev;
      // the overflow pool of a device is keyed by an impossible stream value
      hipStream_t key = on_dev < kMaxPools ? caller : reinterpret_cast<hipStream_t>(~uintptr_t(0));
      for (const Entry& e : pools)
        if (e.dev == dev && e.caller == key) return *e.pool;
      pools.push_back(Entry{dev, key, new Pool()});
      return *pools.back().pool;
    }
  };
  static constexpr int kMaxPools = 16;

  hipStream_t caller_;
  int ns_;
  hipStream_t streams_[kMax] = {};
  Pool* pool_ = nullptr;
  std::unique_lock<std::mutex> lock_;
  hipError_t err_ = hipSuccess;
  bool joined_ = false;
};

// Host-side geometry and diagonal schedule of one problem.
struct DiagPlan {
  int64_t n = 0, nev = 0, NB = 0, K = 0, S = 1, SW = 64;
  int64_t G = 0, M = 0, rows_pad = 0, T = 0;
  std::vector<int> Qm;  // groups of block m

  // SW: columns per stripe (one wave per stripe and tile)
  DiagPlan(int64_t n_, int64_t nev_, int64_t NB_, int64_t K_, int64_t S_, int64_t SW_ = 64)
      : n(n_), nev(nev_), NB(NB_), K(K_), S(S_), SW(SW_) {
    G = (nev + SW - 1) / SW;
    M = (n - 1 + K - 1) / K;
    // deepest row touched: s0 + 1 + (J0-1)*NB + W - 1 < n + NB + K
    rows_pad = ((n + NB + K + 63) / 64) * 64;
    Qm.resize((size_t)M);
    T = 0;
    for (int64_t m = 0; m < M; ++m) {
      const int64_t J0 = (n - 1 - m * K + NB - 1) / NB;
      Qm[(size_t)m] = (int)((J0 + S - 1) / S);
      T = std::max(T, (M - 1 - m) + Qm[(size_t)m]);
    }
  }
  // blocks active at launch t: [m0, m0 + cnt)
  void active(int64_t t, int64_t* m0, int64_t* cnt) const {
    int64_t a = M - 1 - t;
    if (a < 0) a = 0;
    int64_t b = a;
    while (b < M && t - (M - 1 - b) < Qm[(size_t)b]) ++b;
    *m0 = a;
    *cnt = b - a;
  }
  template <typename E>
  size_t qbytes() const {
    return align256((size_t)rows_pad * (size_t)G * (size_t)SW * sizeof(E));
  }
};

// Chase steps per tile.  Model of the launch sequence: a launch of N tiles
// on `slots` resident waves takes ceil(N / slots) rounds, a round costs S + 1
// steps (one step's worth of window load, carry store and wave start per
// tile).  S trades launch tails (fewer, larger tiles) against reload work;
// the S in {1, 2, 3, 4, 6, 8, 12, 16, 24, 32} with the least modelled time
// wins (at n = nev = 20000 it picks 12 for the compact-WY kernel at k = 160,
// measured 340.0 ms against 343.2 at 8 and 341.0 at 16).
inline int64_t choose_steps(int64_t n, int64_t nev, int64_t NB, int64_t K, int64_t slots,
                            int64_t SW) {
  const int64_t G = (nev + SW - 1) / SW;
  const int64_t M = (n - 1 + K - 1) / K;
  if (slots < 1) slots = 1;
  int64_t best = 1;
  double best_cost = -1.0;
  std::vector<int64_t> cnt;
  for (int64_t S : {1, 2, 3, 4, 6, 8, 12, 16, 24, 32}) {
    cnt.assign((size_t)(M + (n - 1 + NB - 1) / NB / S + 2), 0);
    for (int64_t m = 0; m < M; ++m) {
      const int64_t J0 = (n - 1 - m * K + NB - 1) / NB;
      const int64_t Qm = (J0 + S - 1) / S;
      for (int64_t q = 0; q < Qm; ++q) ++cnt[(size_t)((M - 1 - m) + q)];
    }
    double cost = 0.0;
    for (int64_t c : cnt)
      if (c) cost += (double)((G * c + slots - 1) / slots) * (double)(S + 1);
    if (best_cost < 0.0 || cost < best_cost) {
      best_cost = cost;
      best = S;
    }
  }
  return best;
}

// Resident waves of a 64-thread kernel on the whole device.
template <typename F>
int64_t wave_slots(F kernel, int num_cu) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 64, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 4;
  return (int64_t)per_cu * num_cu;
}

}  // namespace ehh
