// Caller-owned device workspaces.
//
// The library allocates no device memory of its own: every plan, factor and
// solve works in a workspace that the caller queries (lsh_*_workspace) and
// passes in.  A handle splits its workspace into Arenas: one for what the
// handle keeps (level matrices, factors, apply vectors) and one or two for
// temporaries that are rewound once per tree level, after the level's work
// is ordered before the next use of the memory.
#include "mem.hpp"

#include <string>

#include "common.hpp"

namespace lsh {
namespace mem {
namespace {
thread_local Arena* g_current = nullptr;
}

void Arena::attach(void* base, size_t cap, const char* what) {
  std::lock_guard<std::mutex> g(mu_);
  base_ = static_cast<char*>(base);
  cap_ = cap;
  top_ = high_ = 0;
  what_ = what;
}

void* Arena::take(size_t bytes) {
  const size_t n = round_up(bytes ? bytes : 1);
  std::lock_guard<std::mutex> g(mu_);
  if (!base_ || top_ + n > cap_)
    throw Error(-7, "workspace too small: the " + what_ + " part needs more than its " + std::to_string(cap_) +
                        " bytes (" + std::to_string(top_) + " in use, " + std::to_string(n) + " more asked)");
  void* p = base_ + top_;
  top_ += n;
  if (top_ > high_) high_ = top_;
  return p;
}

size_t Arena::mark() const {
  std::lock_guard<std::mutex> g(mu_);
  return top_;
}

void Arena::reset(size_t m) {
  std::lock_guard<std::mutex> g(mu_);
  if (m <= top_) top_ = m;
}

size_t Arena::high() const {
  std::lock_guard<std::mutex> g(mu_);
  return high_;
}

Arena* current() { return g_current; }

Bind::Bind(Arena* a) : prev(g_current) { g_current = a; }
Bind::~Bind() { g_current = prev; }

}  // namespace mem
}  // namespace lsh
