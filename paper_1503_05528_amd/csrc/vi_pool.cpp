// vi_pool.cpp -- device memory and timing events reused across contexts.
//
// A context allocates its pyramid, sets, shift maps and scratch at creation
// and releases them when it is destroyed; a server or a benchmark creates and
// destroys contexts of similar sizes over and over.  Going to hipMalloc /
// hipFree each time costs milliseconds per context (the driver maps and
// unmaps the memory), so released blocks are kept per device, by size class,
// and handed to the next request of that class.  The cache is capped
// (VI_POOL_BYTES, default 8 GiB per device); vi_pool_trim returns it to the
// device.  Callers release a block only once no queued work uses it (a
// context synchronises its stream first), so a block may be reused on any
// stream.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdlib>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "vi.h"
#include "vi_internal.h"

namespace vi {
namespace {

struct DevPool {
  std::map<size_t, std::vector<void*>> free;  // size class -> cached blocks
  size_t cached = 0;
  std::vector<hipEvent_t> events;
};

struct Pool {
  std::mutex mu;
  std::map<int, DevPool> dev;
  std::unordered_map<void*, size_t> live;  // block -> size class
  size_t cap = size_t(8) << 30;
};

// Never destroyed: freeing device memory from a static destructor would run
// after the HIP runtime has shut down.
Pool& pool() {
  static Pool* p = [] {
    Pool* q = new Pool();
    if (const char* e = std::getenv("VI_POOL_BYTES")) q->cap = std::strtoull(e, nullptr, 10);
    return q;
  }();
  return *p;
}

// powers of two below 1 MiB, multiples of 2 MiB above
size_t size_class(size_t b) {
  if (b < (size_t(1) << 20)) {
    size_t c = 256;
    while (c < b) c <<= 1;
    return c;
  }
  const size_t g = size_t(2) << 20;
  return (b + g - 1) / g * g;
}

size_t trim_locked(DevPool& d, std::vector<void*>& out) {
  size_t n = 0;
  for (auto& kv : d.free) {
    for (void* p : kv.second) out.push_back(p);
    n += kv.first * kv.second.size();
  }
  d.free.clear();
  d.cached = 0;
  return n;
}

// Failure injection for the tests of the error paths: -1 = off; n >= 0 =
// the next n allocations succeed, every later one fails.
std::atomic<int64_t> g_fail_after{-1};

bool forced_failure() {
  int64_t v = g_fail_after.load();
  while (v >= 0) {
    if (v == 0) return true;
    if (g_fail_after.compare_exchange_weak(v, v - 1)) return false;
  }
  return false;
}

}  // namespace

void* pool_alloc(int dev, size_t bytes) {
  if (forced_failure()) return nullptr;
  Pool& P = pool();
  const size_t cls = size_class(bytes ? bytes : 1);
  {
    std::lock_guard<std::mutex> g(P.mu);
    DevPool& d = P.dev[dev];
    // best fit among cached blocks no more than a quarter larger
    auto it = d.free.lower_bound(cls);
    if (it != d.free.end() && it->first <= cls + cls / 4 && !it->second.empty()) {
      void* p = it->second.back();
      it->second.pop_back();
      d.cached -= it->first;
      P.live[p] = it->first;
      if (it->second.empty()) d.free.erase(it);
      return p;
    }
  }
  void* p = nullptr;
  if (hipMalloc(&p, cls) != hipSuccess) {
    (void)hipGetLastError();
    // give the cache back to the device and try once more
    std::vector<void*> drop;
    {
      std::lock_guard<std::mutex> g(P.mu);
      trim_locked(P.dev[dev], drop);
    }
    for (void* q : drop) (void)hipFree(q);
    p = nullptr;
    if (hipMalloc(&p, cls) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
  }
  std::lock_guard<std::mutex> g(P.mu);
  P.live[p] = cls;
  return p;
}

void pool_free(int dev, void* p) {
  if (!p) return;
  Pool& P = pool();
  bool release = false;
  {
    std::lock_guard<std::mutex> g(P.mu);
    auto it = P.live.find(p);
    if (it == P.live.end()) return;
    const size_t cls = it->second;
    P.live.erase(it);
    DevPool& d = P.dev[dev];
    if (d.cached + cls <= P.cap) {
      d.free[cls].push_back(p);
      d.cached += cls;
    } else {
      release = true;
    }
  }
  if (release) (void)hipFree(p);
}

size_t pool_trim(int dev) {
  Pool& P = pool();
  std::vector<void*> drop;
  size_t n = 0;
  {
    std::lock_guard<std::mutex> g(P.mu);
    n = trim_locked(P.dev[dev], drop);
  }
  for (void* q : drop) (void)hipFree(q);
  return n;
}

hipEvent_t event_get(int dev) {
  Pool& P = pool();
  {
    std::lock_guard<std::mutex> g(P.mu);
    DevPool& d = P.dev[dev];
    if (!d.events.empty()) {
      hipEvent_t e = d.events.back();
      d.events.pop_back();
      return e;
    }
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

void event_put(int dev, hipEvent_t e) {
  if (!e) return;
  Pool& P = pool();
  std::lock_guard<std::mutex> g(P.mu);
  P.dev[dev].events.push_back(e);
}

}  // namespace vi

extern "C" size_t vi_pool_trim(void) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  return vi::pool_trim(dev);
}

extern "C" int64_t vi_debug_fail_allocs(int64_t n) {
  vi::Pool& P = vi::pool();
  int64_t live = 0;
  {
    std::lock_guard<std::mutex> g(P.mu);
    for (const auto& kv : P.live) live += (int64_t)kv.second;
  }
  vi::g_fail_after.store(n < 0 ? -1 : n);
  return live;
}
