// pool.hip -- the library's device memory pool.
//
// Every handle rebuilds its buffers on each Newton step (a new decoupling, a
// new hierarchy, new Krylov workspace), and hipMalloc/hipFree of buffers of
// hundreds of megabytes cost milliseconds, hipFree also synchronising the
// device.  Freed blocks therefore stay cached here and later requests of a
// similar size reuse them; memory goes back to the runtime only through
// rs_pool_trim, or when a hipMalloc fails (the cache is released and the
// allocation retried).
//
// Size classes: powers of two from 256 B to 1 MiB, multiples of 2 MiB above;
// a cached block serves a request if it is at most 1/8 larger.
#include "rs_internal.h"
#include <map>
#include <mutex>
#include <unordered_map>
#include <string.h>

namespace {

struct pool_state {
  std::mutex mu;
  std::multimap<size_t, std::pair<void *, int>> free_blocks;   // size -> (pointer, device)
  std::unordered_map<void *, int> device_of;                    // live and cached blocks
  size_t cached = 0, live = 0;
};

pool_state &pool() {
  static pool_state *p = new pool_state();     // never destroyed: no HIP calls at exit
  return *p;
}

size_t size_class(size_t b) {
  if (b <= ((size_t)1 << 20)) {
    size_t r = 256;
    while (r < b) r <<= 1;
    return r;
  }
  const size_t G = (size_t)2 << 20;
  return (b + G - 1) / G * G;
}

// release every cached block of device dev (-1: all devices); caller holds the lock
void trim_locked(pool_state &P, int dev) {
  for (auto it = P.free_blocks.begin(); it != P.free_blocks.end();) {
    if (dev >= 0 && it->second.second != dev) { ++it; continue; }
    (void)hipFree(it->second.first);
    P.device_of.erase(it->second.first);
    P.cached -= it->first;
    it = P.free_blocks.erase(it);
  }
}

}  // namespace

void *rs_pool_get(size_t bytes, size_t *got) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  const size_t r = size_class(bytes);
  pool_state &P = pool();
  std::lock_guard<std::mutex> lk(P.mu);
  for (auto it = P.free_blocks.lower_bound(r); it != P.free_blocks.end() && it->first <= r + r / 8; ++it) {
    if (it->second.second != dev) continue;
    void *p = it->second.first;
    *got = it->first;
    P.cached -= it->first;
    P.live += it->first;
    P.free_blocks.erase(it);
    return p;
  }
  void *p = nullptr;
  if (hipMalloc(&p, r) != hipSuccess) {
    (void)hipGetLastError();
    trim_locked(P, dev);
    p = nullptr;
    if (hipMalloc(&p, r) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
  }
  P.device_of[p] = dev;
  P.live += r;
  *got = r;
  return p;
}

void rs_pool_put(void *p, size_t bytes) {
  if (!p) return;
  pool_state &P = pool();
  std::lock_guard<std::mutex> lk(P.mu);
  auto d = P.device_of.find(p);
  int dev = d == P.device_of.end() ? 0 : d->second;
  P.free_blocks.emplace(bytes, std::make_pair(p, dev));
  P.live -= bytes;
  P.cached += bytes;
}

extern "C" void rs_pool_trim(void) {
  pool_state &P = pool();
  std::lock_guard<std::mutex> lk(P.mu);
  trim_locked(P, -1);
}

extern "C" void rs_pool_usage(size_t *live_bytes, size_t *cached_bytes) {
  pool_state &P = pool();
  std::lock_guard<std::mutex> lk(P.mu);
  if (live_bytes) *live_bytes = P.live;
  if (cached_bytes) *cached_bytes = P.cached;
}

// ---- short host waits --------------------------------------------------------
// The set-up reads a few counts and flags back (an aggregate count, an error
// word) and waits for the stream at each.  A blocking stream synchronisation
// leaves the device idle for tens of microseconds after such a read while the
// host thread wakes up; these waits poll an event instead.  Each host thread
// keeps one event per device and a small pinned staging buffer (never freed:
// no HIP calls at exit).
namespace {
constexpr int WAIT_MAX_DEV = 64;
constexpr size_t WAIT_STAGE = 256;
struct host_wait {
  hipEvent_t ev[WAIT_MAX_DEV] = {};
  void *stage = nullptr;
};
thread_local host_wait tw;
}  // namespace

rs_status rs_wait(hipStream_t s) {
  int dev = 0;
  RS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= WAIT_MAX_DEV) {
    RS_HIP(hipStreamSynchronize(s));
    return RS_OK;
  }
  if (!tw.ev[dev]) RS_HIP(hipEventCreateWithFlags(&tw.ev[dev], hipEventDisableTiming));
  RS_HIP(hipEventRecord(tw.ev[dev], s));
  for (;;) {
    const hipError_t e = hipEventQuery(tw.ev[dev]);
    if (e == hipSuccess) return RS_OK;
    if (e != hipErrorNotReady) return RS_E_HIP;
  }
}

rs_status rs_wait_read(void *h, const void *d, size_t bytes, hipStream_t s) {
  if (bytes > WAIT_STAGE) {
    RS_HIP(hipMemcpyAsync(h, d, bytes, hipMemcpyDeviceToHost, s));
    RS_HIP(hipStreamSynchronize(s));
    return RS_OK;
  }
  if (!tw.stage) RS_HIP(hipHostMalloc(&tw.stage, WAIT_STAGE, hipHostMallocPortable));
  RS_HIP(hipMemcpyAsync(tw.stage, d, bytes, hipMemcpyDeviceToHost, s));
  RS_TRY(rs_wait(s));
  memcpy(h, tw.stage, bytes);
  return RS_OK;
}
