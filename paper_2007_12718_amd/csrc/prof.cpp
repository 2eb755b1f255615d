// Per-kernel hipEvent timing store (see prof.hpp).
#include "prof.hpp"

#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

namespace lsh {
namespace prof {
namespace {
struct Rec {
  std::string name;
  hipEvent_t a = nullptr, b = nullptr;
  hipStream_t s = nullptr;
  double work = 0, bytes = 0;
};
std::mutex mu;
bool on = false;
std::string only;  // record only names starting with this (empty: all)
std::vector<Rec> recs;
std::vector<hipEvent_t> pool;
hipEvent_t get_event() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

bool enabled() { return on; }

void record(const char* name, hipStream_t s, double work, double bytes, bool start) {
  std::lock_guard<std::mutex> g(mu);
  if (!only.empty() && std::strncmp(name, only.c_str(), only.size()) != 0) return;
  if (start) {
    Rec r;
    r.name = name;
    r.work = work;
    r.bytes = bytes;
    r.s = s;
    r.a = get_event();
    if (r.a) (void)hipEventRecord(r.a, s);
    recs.push_back(r);
  } else {
    for (auto it = recs.rbegin(); it != recs.rend(); ++it)
      if (it->b == nullptr && it->s == s && it->name == name) {
        it->b = get_event();
        if (it->b) (void)hipEventRecord(it->b, s);
        break;
      }
  }
}

void set(bool enable) {
  std::lock_guard<std::mutex> g(mu);
  for (auto& r : recs) {
    if (r.a) pool.push_back(r.a);
    if (r.b) pool.push_back(r.b);
  }
  recs.clear();
  on = enable;
  // events are created ahead so that recording costs one hipEventRecord
  while (enable && pool.size() < 8192) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) break;
    pool.push_back(e);
  }
}

void set_only(const char* prefix) {
  std::lock_guard<std::mutex> g(mu);
  only = prefix ? prefix : "";
}

// totals per kernel name: launches, ms, work, algorithmic bytes
int query(const char* name, int* launches, double* ms, double* work, double* bytes) {
  std::lock_guard<std::mutex> g(mu);
  (void)hipDeviceSynchronize();
  int n = 0;
  double t = 0, w = 0, by = 0;
  for (auto& r : recs) {
    if (r.name != name || !r.a || !r.b) continue;
    float e = 0;
    if (hipEventElapsedTime(&e, r.a, r.b) == hipSuccess) t += e;
    w += r.work;
    by += r.bytes;
    ++n;
  }
  if (launches) *launches = n;
  if (ms) *ms = t;
  if (work) *work = w;
  if (bytes) *bytes = by;
  return 0;
}

// distinct names recorded so far, separated by ';'
std::string names() {
  std::lock_guard<std::mutex> g(mu);
  std::map<std::string, int> m;
  for (auto& r : recs) m[r.name]++;
  std::string s;
  for (auto& kv : m) {
    if (!s.empty()) s += ";";
    s += kv.first;
  }
  return s;
}
}  // namespace prof
}  // namespace lsh
