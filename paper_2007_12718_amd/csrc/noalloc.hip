// lsh_dev_inverse_static: the batched Gauss-Jordan inverse of lsh_dev_inverse
// with its scratch in a static device array instead of a caller workspace,
// for callers that cannot allocate device memory at all.
//
// `scratch` is a file-scope device array, one copy per GPU, held for the
// life of the process.  In host code its name is only a stand-in for the
// symbol: its device address is looked up once per device with
// hipGetSymbolAddress (with that device current) and kept; the kernels get
// that address, never the name.  Every call on a GPU shares that GPU's copy,
// so calls that overlap on one GPU (other streams, other host threads) race;
// the inverse's kernels initialise every part of the scratch they read.
#include <mutex>

#include "../../include/lsh_dev.h"
#include "blas.hpp"

namespace {

constexpr size_t kStaticScratchBytes = size_t(32) << 20;
static __device__ __align__(256) char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices] = {};

// device address of this device's scratch (looked up on first use, with the
// device current)
void* scratch_address() {
  int dev = 0;
  LSH_HIP(hipGetDevice(&dev));
  LSH_REQUIRE(dev >= 0 && dev < kMaxDevices, LSH_ERR_UNSUPPORTED, "device index beyond the static scratch table");
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_addr[dev]) {
    void* p = nullptr;
    LSH_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    LSH_REQUIRE(p != nullptr, LSH_ERR_HIP, "no device address for the static scratch");
    g_addr[dev] = p;
  }
  return g_addr[dev];
}

}  // namespace

namespace lsh {
// message of the last failure (defined with the other entry points)
int report_failure(const Error& e);
int report_other_failure(const std::exception& e);
}  // namespace lsh

extern "C" int lsh_dev_inverse_static(int prec, void* A, int c, long lda, long sA, int batch, int* info,
                                      void* stream) {
  try {
    LSH_REQUIRE(A && c >= 1 && batch >= 1 && lda >= c, LSH_ERR_INVALID_ARG, "bad inverse argument");
    const size_t need =
        prec == LSH_FP64 ? lsh::inverse_ws_bytes<double>(c, batch) : lsh::inverse_ws_bytes<float>(c, batch);
    LSH_REQUIRE(need <= kStaticScratchBytes, LSH_ERR_WORKSPACE_TOO_SMALL,
                "lsh_dev_inverse_static: " + std::to_string(batch) + " matrices of order " + std::to_string(c) +
                    " need " + std::to_string(need) + " bytes of scratch; the static scratch holds " +
                    std::to_string(kStaticScratchBytes));
    void* ws = scratch_address();
    hipStream_t s = (hipStream_t)stream;
    if (prec == LSH_FP64) lsh::inverse<double>(s, (lsh::z64*)A, c, lda, sA, batch, ws, info);
    else lsh::inverse<float>(s, (lsh::c32*)A, c, lda, sA, batch, ws, info);
    return LSH_OK;
  } catch (const lsh::Error& e) {
    return lsh::report_failure(e);
  } catch (const std::exception& e) {
    return lsh::report_other_failure(e);
  }
}
