// Process-wide cache of per-level compression data (see plancache.cpp).
#pragma once
#include <cstdint>
#include <vector>

#include "common.hpp"
#include "hbs.hpp"

namespace lsh {
namespace pcache {

// What a row ID depends on: the box (its size fixes the candidate geometry
// and the proxy ring), kappa h, the tolerance, the ring width, the matrix
// order and the pivoting method.  The IDs do not depend on h itself (the
// table scales as h^2, which moves neither the pivots nor U).
struct Key {
  int dev = 0, kind = 0;  // kind 0: level row ID; 1: sibling block row ID
  int sx = 0, sy = 0, w = 0, order = 0, method = 0;
  uint64_t kh = 0, tol = 0, alpha = 0;
  bool operator<(const Key& o) const;
};

// Looks up key; rows (the points the ID was taken over, identifying the
// entry) must equal the cached ones.  On a hit, J and k are set and U
// (m x k, FP64, m as stored) is copied into a new buffer from the bound
// arena on stream s (the call synchronises s).
bool find(const Key& key, const std::vector<I2>& rows, std::vector<int>& J, int& k, DevBuf& U, hipStream_t s);
// Stores a host copy of the m x k matrix U (copied on stream s; the call
// synchronises s).
void insert(const Key& key, const std::vector<I2>& rows, const std::vector<int>& J, int m, int k, const DevBuf& U,
            hipStream_t s);
void clear();
void info(int* entries, size_t* bytes);
// Binary file of every entry (host copies); load adds the file's entries
// for the current device, replacing equal keys.
void save(const char* path);
void load(const char* path);

}  // namespace pcache
}  // namespace lsh
