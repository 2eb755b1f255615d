// Wave-level reductions on DPP lane exchanges (device code; included by the
// kernel sources only).
#pragma once
#include <hip/hip_runtime.h>

namespace lsh {

// Wave-wide maximum of a 32-bit key, the same in every lane: DPP exchanges
// inside each 16-lane row (quad butterflies, then the half-row and row
// mirrors), then the four row maxima through readlane.
template <int CTRL>
__device__ __forceinline__ unsigned dpp_max_u32(unsigned k) {
  const unsigned o = (unsigned)__builtin_amdgcn_update_dpp(0, (int)k, CTRL, 0xF, 0xF, false);
  return o > k ? o : k;
}
__device__ __forceinline__ unsigned wave_max_u32_uniform(unsigned k) {
  k = dpp_max_u32<0xB1>(k);   // quad_perm [1,0,3,2]
  k = dpp_max_u32<0x4E>(k);   // quad_perm [2,3,0,1]
  k = dpp_max_u32<0x141>(k);  // row_half_mirror
  k = dpp_max_u32<0x140>(k);  // row_mirror
  unsigned best = (unsigned)__builtin_amdgcn_readlane((int)k, 0);
#pragma unroll
  for (int r = 1; r < 4; ++r) {
    const unsigned v = (unsigned)__builtin_amdgcn_readlane((int)k, 16 * r);
    best = v > best ? v : best;
  }
  return best;
}

}  // namespace lsh
