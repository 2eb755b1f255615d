// Device-memory cache for the buffers that plans and factors own.
//
// hipFree synchronises the device and unmaps the pages, and a fresh hipMalloc
// maps new ones: for a factor of a few hundred buffers that costs tens of
// milliseconds per build/destroy cycle.  Destroying a plan or factor first
// synchronises the device once (after which nothing in flight can use its
// memory) and then hands every buffer to this cache; the next allocation of
// a similar size on the same device takes it back without a runtime call.
// The cache holds at most kCap bytes (LSH_CACHE_BYTES overrides; 0 turns it
// off); a failed hipMalloc empties it and retries once.
#include "mem.hpp"

#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <utility>

namespace lsh {
namespace mem {
namespace {
std::mutex mu;
std::multimap<std::pair<int, size_t>, void*> blocks;  // (device, capacity) -> pointer
size_t held = 0;
thread_local int recycle_depth = 0;

bool trace() {
  static const bool t = [] {
    const char* e = std::getenv("LSH_MEM_TRACE");
    return e && *e == '1';
  }();
  return t;
}

size_t cap_bytes() {
  static const size_t c = [] {
    const char* e = std::getenv("LSH_CACHE_BYTES");
    if (e && *e) return (size_t)std::strtoull(e, nullptr, 10);
    return (size_t)32 << 30;
  }();
  return c;
}

// Capacities are rounded so that the sizes of one workload land on a few
// classes: 256 B granules below 1 MiB, 64 KiB granules above.
size_t round_cap(size_t n) {
  const size_t g = n < (1u << 20) ? 256 : (64u << 10);
  return (n + g - 1) / g * g;
}

void free_all_locked() {
  for (auto& kv : blocks) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != kv.first.first) (void)hipSetDevice(kv.first.first);
    (void)hipFree(kv.second);
    if (cur != kv.first.first) (void)hipSetDevice(cur);
  }
  blocks.clear();
  held = 0;
}
}  // namespace

hipError_t get(size_t n, void** p, size_t* cap) {
  *p = nullptr;
  *cap = round_cap(n);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  {
    std::lock_guard<std::mutex> g(mu);
    // smallest cached block of at least the rounded size, at most 1/8 larger
    auto it = blocks.lower_bound({dev, *cap});
    if (it != blocks.end() && it->first.first == dev && it->first.second <= *cap + *cap / 8) {
      *p = it->second;
      *cap = it->first.second;
      held -= *cap;
      blocks.erase(it);
      return hipSuccess;
    }
  }
  if (trace()) std::fprintf(stderr, "lsh mem: hipMalloc %zu bytes (cache miss)\n", *cap);
  e = hipMalloc(p, *cap);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    {
      std::lock_guard<std::mutex> g(mu);
      if (blocks.empty()) return e;
      (void)hipDeviceSynchronize();
      free_all_locked();
    }
    e = hipMalloc(p, *cap);
  }
  return e;
}

void put(void* p, size_t cap) {
  if (!p) return;
  if (recycle_depth > 0 && cap_bytes() > 0) {
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
      std::lock_guard<std::mutex> g(mu);
      if (held + cap <= cap_bytes()) {
        blocks.insert({{dev, cap}, p});
        held += cap;
        return;
      }
    }
  }
  if (trace()) std::fprintf(stderr, "lsh mem: hipFree %zu bytes (outside a destroy)\n", cap);
  (void)hipFree(p);
}

Recycle::Recycle() {
  (void)hipDeviceSynchronize();
  ++recycle_depth;
}
Recycle::~Recycle() { --recycle_depth; }

void trim() {
  std::lock_guard<std::mutex> g(mu);
  (void)hipDeviceSynchronize();
  free_all_locked();
}

size_t cached_bytes() {
  std::lock_guard<std::mutex> g(mu);
  return held;
}
}  // namespace mem
}  // namespace lsh
