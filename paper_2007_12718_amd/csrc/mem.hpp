// Device-memory cache behind DevBuf (see mem.cpp).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

namespace lsh {
namespace mem {
// A block of at least n bytes on the current device (its capacity in *cap).
hipError_t get(size_t n, void** p, size_t* cap);
// Returns a block: into the cache inside a Recycle scope, else hipFree.
void put(void* p, size_t cap);
// Synchronises the device on entry; DevBuf releases inside the scope (on this
// thread) go to the cache, which is safe because no work is in flight.
struct Recycle {
  Recycle();
  ~Recycle();
  Recycle(const Recycle&) = delete;
  Recycle& operator=(const Recycle&) = delete;
};
// Frees every cached block (synchronises the device).
void trim();
size_t cached_bytes();
}  // namespace mem
}  // namespace lsh
