// Workspace cache of the back-transformation calls.
//
// Every call needs a device workspace for the duration of its launches (the
// stripe-major copy of Q and the packed reflectors, up to a few GB).  The
// cache keeps freed blocks per device and hands one out again when it is
// large enough and no pending work uses it: to the stream that freed it at
// once (stream order protects it), to another stream only after the event
// recorded behind its last use has completed.  A call never waits for work on
// another stream to reuse memory, so calls on different streams overlap; a
// stream-ordered allocator that makes the second stream wait for the first
// one's work to reuse a block would run them one after the other.
//
// Blocks are hipMalloc'd in 2 MiB multiples, and a block serves requests of
// at least half its size.  Idle blocks beyond kKeepBytes per device are freed,
// least recently used first, before a new block is allocated, and all idle
// blocks are freed when an allocation fails or on elpa_hh_workspace_release.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <vector>

#include "../../include/elpa_hh.h"
#include "hh_sched.h"

namespace ehh {
namespace {

constexpr size_t kGrain = size_t(2) << 20;
constexpr size_t kKeepBytes = size_t(8) << 30;

struct Block {
  int dev;
  void* p;
  size_t bytes;
  bool busy;
  hipStream_t last;      // stream of the last use
  hipEvent_t ev;         // recorded on `last` behind the last use
  uint64_t tick;         // last release, for least-recently-used eviction
};

struct Cache {
  std::mutex mu;
  std::vector<Block> blocks;
  uint64_t tick = 0;
  std::vector<size_t> total;  // device memory per device id (0: unknown)

  static Cache& get() {
    static Cache c;
    return c;
  }

  // idle: not handed out and no pending work uses it (as seen from `st`)
  static bool idle_for(const Block& b, hipStream_t st) {
    if (b.busy) return false;
    if (!b.ev || b.last == st) return true;
    return hipEventQuery(b.ev) == hipSuccess;
  }

  // Frees idle blocks of `dev` whose last use has completed, least recently
  // used first, until the idle bytes are at most `keep`.  Returns the bytes
  // freed.  Called with mu held.
  size_t evict(int dev, size_t keep) {
    size_t idle = 0;
    for (const Block& b : blocks)
      if (b.dev == dev && !b.busy) idle += b.bytes;
    size_t freed = 0;
    while (idle > keep) {
      int pick = -1;
      for (int i = 0; i < (int)blocks.size(); ++i) {
        const Block& b = blocks[(size_t)i];
        if (b.dev != dev || b.busy || (b.ev && hipEventQuery(b.ev) != hipSuccess)) continue;
        if (pick < 0 || b.tick < blocks[(size_t)pick].tick) pick = i;
      }
      if (pick < 0) break;
      Block b = blocks[(size_t)pick];
      blocks.erase(blocks.begin() + pick);
      (void)hipFree(b.p);
      if (b.ev) (void)hipEventDestroy(b.ev);
      idle -= b.bytes;
      freed += b.bytes;
    }
    (void)hipGetLastError();
    return freed;
  }
};

}  // namespace

hipError_t ws_alloc(void** p, size_t bytes, hipStream_t st) {
  *p = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  Cache& c = Cache::get();
  {
    std::lock_guard<std::mutex> g(c.mu);
    if ((size_t)dev >= c.total.size()) c.total.resize((size_t)dev + 1, 0);
    if (c.total[(size_t)dev] == 0) {
      size_t t = 0;
      if (hipDeviceTotalMem(&t, dev) == hipSuccess) c.total[(size_t)dev] = t;
    }
    if (c.total[(size_t)dev] != 0 && bytes > c.total[(size_t)dev]) return hipErrorOutOfMemory;
  }
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  e = hipStreamIsCapturing(st, &cs);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return e;
  }
  if (cs != hipStreamCaptureStatusNone) {
    // a graph owns what is allocated while it is captured
    e = hipMallocAsync(p, bytes, st);
    if (e != hipSuccess) (void)hipGetLastError();
    return e;
  }
  const size_t need = bytes == 0 ? kGrain : (bytes + kGrain - 1) / kGrain * kGrain;
  {
    std::lock_guard<std::mutex> g(c.mu);
    int pick = -1;
    for (int i = 0; i < (int)c.blocks.size(); ++i) {
      const Block& b = c.blocks[(size_t)i];
      if (b.dev != dev || b.bytes < need || b.bytes / 2 > need || !Cache::idle_for(b, st))
        continue;
      if (pick < 0 || b.bytes < c.blocks[(size_t)pick].bytes) pick = i;
    }
    if (pick >= 0) {
      Block& b = c.blocks[(size_t)pick];
      b.busy = true;
      *p = b.p;
      return hipSuccess;
    }
    c.evict(dev, kKeepBytes > need ? kKeepBytes - need : 0);
  }
  void* q = nullptr;
  e = hipMalloc(&q, need);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    {
      std::lock_guard<std::mutex> g(c.mu);
      c.evict(dev, 0);
    }
    e = hipMalloc(&q, need);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return e;
    }
  }
  std::lock_guard<std::mutex> g(c.mu);
  c.blocks.push_back(Block{dev, q, need, true, st, nullptr, ++c.tick});
  *p = q;
  return hipSuccess;
}

hipError_t ws_free(void* p, hipStream_t st) {
  if (!p) return hipSuccess;
  Cache& c = Cache::get();
  std::lock_guard<std::mutex> g(c.mu);
  for (Block& b : c.blocks) {
    if (b.p != p || !b.busy) continue;
    hipError_t e = hipSuccess;
    if (!b.ev) e = hipEventCreateWithFlags(&b.ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(b.ev, st);
    if (e != hipSuccess) {
      // without an event the block's last use cannot be told: keep it out
      // of circulation until it is released explicitly
      (void)hipGetLastError();
      return e;
    }
    b.last = st;
    b.busy = false;
    b.tick = ++c.tick;
    return hipSuccess;
  }
  // not a cache block: a graph-owned allocation made during capture
  return hipFreeAsync(p, st);
}

size_t ws_cached_bytes(int dev) {
  Cache& c = Cache::get();
  std::lock_guard<std::mutex> g(c.mu);
  size_t s = 0;
  for (const Block& b : c.blocks)
    if (b.dev == dev) s += b.bytes;
  return s;
}

size_t ws_release(int dev) {
  Cache& c = Cache::get();
  std::lock_guard<std::mutex> g(c.mu);
  return c.evict(dev, 0);
}

}  // namespace ehh

extern "C" {

int64_t elpa_hh_workspace_cached(void) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return ELPA_ERR_DEVICE;
  return (int64_t)ehh::ws_cached_bytes(dev);
}

int64_t elpa_hh_workspace_release(void) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return ELPA_ERR_DEVICE;
  return (int64_t)ehh::ws_release(dev);
}

}  // extern "C"
