// Shared device/host helpers for the HBS Lippmann-Schwinger library (gfx950).
#pragma once
#include <hip/hip_runtime.h>

#include "mem.hpp"

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

namespace lsh {

// Interleaved complex number in the working precision R (float or double).
template <typename R>
struct alignas(2 * sizeof(R)) cplx {
  R x, y;
};

template <typename R>
__host__ __device__ inline cplx<R> mk(R a, R b) {
  cplx<R> z;
  z.x = a;
  z.y = b;
  return z;
}
template <typename R>
__host__ __device__ inline cplx<R> operator+(cplx<R> a, cplx<R> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename R>
__host__ __device__ inline cplx<R> operator-(cplx<R> a, cplx<R> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename R>
__host__ __device__ inline cplx<R> operator*(cplx<R> a, cplx<R> b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename R>
__host__ __device__ inline cplx<R> operator*(R s, cplx<R> a) { return mk(s * a.x, s * a.y); }
template <typename R>
__host__ __device__ inline cplx<R> conjg(cplx<R> a) { return mk(a.x, -a.y); }
template <typename R>
__host__ __device__ inline R abs2(cplx<R> a) { return a.x * a.x + a.y * a.y; }
// a += b * c
template <typename R>
__host__ __device__ inline void fma_acc(cplx<R>& a, cplx<R> b, cplx<R> c) {
  a.x += b.x * c.x - b.y * c.y;
  a.y += b.x * c.y + b.y * c.x;
}
template <typename R>
__host__ __device__ inline cplx<R> cdiv(cplx<R> a, cplx<R> b) {
  R d = b.x * b.x + b.y * b.y;
  return mk((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
template <typename R>
__host__ __device__ inline cplx<R> crecip(cplx<R> b) {
  R d = b.x * b.x + b.y * b.y;
  return mk(b.x / d, -b.y / d);
}

using z64 = cplx<double>;
using c32 = cplx<float>;

// Library error: carries a status code and a message for lsh_last_error().
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define LSH_HIP(call)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      throw ::lsh::Error(-4, std::string(#call) + ": " + hipGetErrorString(e_) + " at " + \
                                 __FILE__ + ":" + std::to_string(__LINE__));             \
  } while (0)

#define LSH_REQUIRE(cond, code, msg)                      \
  do {                                                    \
    if (!(cond)) throw ::lsh::Error((code), std::string(msg)); \
  } while (0)

#define LSH_LAUNCH_CHECK() LSH_HIP(hipGetLastError())

// Device memory carved from a caller-owned workspace: alloc() takes from the
// arena bound to the calling thread (mem::Bind) or from a given arena;
// release() only forgets the pointer (the arena rewinds as a whole).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  explicit DevBuf(size_t n) { alloc(n); }
  void alloc(size_t n) {
    mem::Arena* a = mem::current();
    if (n && !a) throw Error(-1, "internal: device allocation outside a workspace");
    alloc_in(*a, n);
  }
  void alloc_in(mem::Arena& a, size_t n) {
    bytes = n;
    p = n ? a.take(n) : nullptr;
  }
  void release() {
    p = nullptr;
    bytes = 0;
  }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      p = o.p; bytes = o.bytes;
      o.p = nullptr; o.bytes = 0;
    }
    return *this;
  }
  template <typename T>
  T* as() const { return static_cast<T*>(p); }
};

inline int ceil_div(long a, long b) { return int((a + b - 1) / b); }

}  // namespace lsh
