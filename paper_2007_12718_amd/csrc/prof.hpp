// Per-kernel hipEvent timing (off by default): each instrumented launch
// records a start/stop event pair on its own stream plus the launch's
// algorithmic work (flops or bytes, as the launcher defines it).  Names that
// start with "op_" cover a composite operation (several kernels).
#pragma once
#include <hip/hip_runtime.h>

namespace lsh {
namespace prof {
bool enabled();
void record(const char* name, hipStream_t s, double work, double bytes, bool start);
}  // namespace prof

// bytes (optional): the launch's algorithmic memory traffic where work counts flops
struct ProfScope {
  const char* name;
  hipStream_t s;
  double work, bytes;
  bool on;
  ProfScope(const char* n, hipStream_t st, double w, double by = 0)
      : name(n), s(st), work(w), bytes(by), on(prof::enabled()) {
    if (on) prof::record(name, s, work, bytes, true);
  }
  ~ProfScope() {
    if (on) prof::record(name, s, work, bytes, false);
  }
};
}  // namespace lsh
