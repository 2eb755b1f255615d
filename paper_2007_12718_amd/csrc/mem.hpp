// Caller-owned device workspaces (see mem.cpp).
#pragma once
#include <cstddef>
#include <mutex>
#include <string>

namespace lsh {
namespace mem {

constexpr size_t kGranule = 256;
inline size_t round_up(size_t n) { return (n + kGranule - 1) / kGranule * kGranule; }

// A region of a caller's device workspace, handed out by bumping an offset
// in 256-byte granules.  Nothing is returned piecemeal: reset() rewinds to a
// mark once the work that used the memory after it is ordered before the
// next use (same stream, or synchronised).  Running out throws
// LSH_ERR_WORKSPACE_TOO_SMALL.  Thread-safe.
class Arena {
 public:
  void attach(void* base, size_t cap, const char* what);
  void* take(size_t bytes);
  size_t mark() const;
  void reset(size_t mark);
  size_t cap() const { return cap_; }
  size_t high() const;  // high-water mark (bytes)
  char* base() const { return base_; }

 private:
  char* base_ = nullptr;
  size_t cap_ = 0, top_ = 0, high_ = 0;
  std::string what_;
  mutable std::mutex mu_;
};

// Byte count of a sequence of takes (the same rounding as Arena::take).
struct Sizer {
  size_t total = 0;
  void add(size_t bytes) { total += round_up(bytes ? bytes : 1); }
  template <typename T>
  void add_n(size_t count) { add(sizeof(T) * count); }
};

// The arena that DevBuf::alloc draws from on the calling thread.
Arena* current();
struct Bind {
  explicit Bind(Arena* a);
  ~Bind();
  Bind(const Bind&) = delete;
  Bind& operator=(const Bind&) = delete;
  Arena* prev;
};

}  // namespace mem
}  // namespace lsh
