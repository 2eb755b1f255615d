// Process-wide cache of per-level compression data: the row IDs of the
// universal (b-independent) compression, Sec. 3.2, depend only on the box
// size, kappa h, the tolerance, the ring width, the matrix order and the
// pivoting rule, so one plan's levels serve later plans, on other b and on
// other grids with the same kappa h.  Entries live in host memory (the
// library owns no device memory): candidates, pivots and U; a hit copies U
// into the plan's workspace.
#include "plancache.hpp"

#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>

namespace lsh {
namespace pcache {

bool Key::operator<(const Key& o) const {
  return std::tie(dev, kind, sx, sy, w, order, method, kh, tol, alpha) <
         std::tie(o.dev, o.kind, o.sx, o.sy, o.w, o.order, o.method, o.kh, o.tol, o.alpha);
}

namespace {
struct Entry {
  std::vector<I2> rows;
  std::vector<int> J;
  int m = 0, k = 0;
  std::vector<z64> U;  // m x k, row-major
};
std::mutex mu;
std::map<Key, std::shared_ptr<Entry>> entries;

bool same_rows(const std::vector<I2>& a, const std::vector<I2>& b) {
  if (a.size() != b.size()) return false;
  for (size_t i = 0; i < a.size(); ++i)
    if (a[i].x != b[i].x || a[i].y != b[i].y) return false;
  return true;
}
}  // namespace

bool find(const Key& key, const std::vector<I2>& rows, std::vector<int>& J, int& k, DevBuf& U, hipStream_t s) {
  std::shared_ptr<Entry> e;
  {
    std::lock_guard<std::mutex> g(mu);
    auto it = entries.find(key);
    if (it == entries.end()) return false;
    e = it->second;
  }
  if (!same_rows(e->rows, rows)) return false;
  J = e->J;
  k = e->k;
  const size_t bytes = sizeof(z64) * (size_t)e->m * e->k;
  U.alloc(bytes);
  LSH_HIP(hipMemcpyAsync(U.p, e->U.data(), bytes, hipMemcpyHostToDevice, s));
  LSH_HIP(hipStreamSynchronize(s));  // (the entry is held by e until here)
  return true;
}

void insert(const Key& key, const std::vector<I2>& rows, const std::vector<int>& J, int m, int k, const DevBuf& U,
            hipStream_t s) {
  auto e = std::make_shared<Entry>();
  e->rows = rows;
  e->J = J;
  e->m = m;
  e->k = k;
  const size_t bytes = sizeof(z64) * (size_t)m * k;
  LSH_REQUIRE((int)J.size() == k && U.bytes >= bytes, -1, "plan cache: inconsistent entry");
  e->U.resize((size_t)m * k);
  LSH_HIP(hipMemcpyAsync(e->U.data(), U.p, bytes, hipMemcpyDeviceToHost, s));
  LSH_HIP(hipStreamSynchronize(s));
  std::lock_guard<std::mutex> g(mu);
  entries[key] = e;
}

void clear() {
  std::map<Key, std::shared_ptr<Entry>> old;
  {
    std::lock_guard<std::mutex> g(mu);
    old.swap(entries);
  }
}

void info(int* n, size_t* bytes) {
  std::lock_guard<std::mutex> g(mu);
  size_t b = 0;
  for (auto& kv : entries) b += sizeof(z64) * kv.second->U.size();
  if (n) *n = (int)entries.size();
  if (bytes) *bytes = b;
}

namespace {
const char kMagic[8] = {'L', 'S', 'H', 'P', 'C', 'A', 'C', '1'};
struct FileCloser {
  FILE* f;
  ~FileCloser() { if (f) std::fclose(f); }
};
void put(FILE* f, const void* p, size_t n) {
  LSH_REQUIRE(std::fwrite(p, 1, n, f) == n, -1, "plan cache: write failed");
}
void get(FILE* f, void* p, size_t n) {
  LSH_REQUIRE(std::fread(p, 1, n, f) == n, -1, "plan cache: truncated file");
}
}  // namespace

// Layout: magic, entry count (int64), then per entry the Key (with dev
// rewritten on load), m, k, the row count nr, rows (nr x I2), J (k ints),
// U (m x k double2).
void save(const char* path) {
  std::vector<std::pair<Key, std::shared_ptr<Entry>>> all;
  {
    std::lock_guard<std::mutex> g(mu);
    for (auto& kv : entries) all.push_back(kv);
  }
  FileCloser fc{std::fopen(path, "wb")};
  LSH_REQUIRE(fc.f, -1, std::string("plan cache: cannot open ") + path);
  put(fc.f, kMagic, sizeof(kMagic));
  const int64_t n = (int64_t)all.size();
  put(fc.f, &n, sizeof(n));
  for (auto& kv : all) {
    const Entry& e = *kv.second;
    put(fc.f, &kv.first, sizeof(Key));
    const int nr = (int)e.rows.size();
    put(fc.f, &e.m, sizeof(int));
    put(fc.f, &e.k, sizeof(int));
    put(fc.f, &nr, sizeof(int));
    put(fc.f, e.rows.data(), sizeof(I2) * e.rows.size());
    put(fc.f, e.J.data(), sizeof(int) * e.J.size());
    put(fc.f, e.U.data(), sizeof(z64) * e.U.size());
  }
}

void load(const char* path) {
  FileCloser fc{std::fopen(path, "rb")};
  LSH_REQUIRE(fc.f, -1, std::string("plan cache: cannot open ") + path);
  char magic[8];
  get(fc.f, magic, sizeof(magic));
  LSH_REQUIRE(std::memcmp(magic, kMagic, sizeof(magic)) == 0, -1, "plan cache: not a plan cache file");
  int64_t n = 0;
  get(fc.f, &n, sizeof(n));
  LSH_REQUIRE(n >= 0 && n < (1 << 20), -1, "plan cache: bad entry count");
  int dev = 0;
  LSH_HIP(hipGetDevice(&dev));
  for (int64_t q = 0; q < n; ++q) {
    Key key;
    get(fc.f, &key, sizeof(Key));
    auto e = std::make_shared<Entry>();
    int nr = 0;
    get(fc.f, &e->m, sizeof(int));
    get(fc.f, &e->k, sizeof(int));
    get(fc.f, &nr, sizeof(int));
    LSH_REQUIRE(e->m >= 1 && e->k >= 1 && e->k <= e->m && e->m <= (1 << 16) && nr >= 1 && nr <= (1 << 17), -1,
                "plan cache: bad entry size");
    e->rows.resize(nr);
    e->J.resize(e->k);
    get(fc.f, e->rows.data(), sizeof(I2) * nr);
    get(fc.f, e->J.data(), sizeof(int) * e->k);
    for (int j : e->J) LSH_REQUIRE(j >= 0 && j < e->m, -1, "plan cache: bad pivot index");
    e->U.resize((size_t)e->m * e->k);
    get(fc.f, e->U.data(), sizeof(z64) * e->U.size());
    key.dev = dev;
    std::lock_guard<std::mutex> g(mu);
    entries[key] = e;
  }
}

}  // namespace pcache
}  // namespace lsh
