// Per-kernel hipEvent timing (off by default): each instrumented launch
// records a start/stop event pair on its own stream plus the launch's
// algorithmic work (flops or bytes, as the launcher defines it).  Names that
// start with "op_" cover a composite operation (several kernels).
#pragma once
#include <hip/hip_runtime.h>

namespace lsh {
namespace prof {
bool enabled();
void record(const char* name, hipStream_t s, double work, bool start);
}  // namespace prof

struct ProfScope {
  const char* name;
  hipStream_t s;
  double work;
  bool on;
  ProfScope(const char* n, hipStream_t st, double w) : name(n), s(st), work(w), on(prof::enabled()) {
    if (on) prof::record(name, s, work, true);
  }
  ~ProfScope() {
    if (on) prof::record(name, s, work, false);
  }
};
}  // namespace lsh
