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

// DPP lane exchange of a float or double (CTRL: a DPP control inside a
// 16-lane row), and the sum over groups of L lanes, the same in every lane of
// a group: DPP butterflies inside rows of 16, then exchanges across rows.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <int L, typename R>
__device__ __forceinline__ R group_sum(R v) {
  if (L >= 2) v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]
  if (L >= 4) v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]
  if (L >= 8) v += dpp_mov<0x141>(v);  // row_half_mirror
  if (L >= 16) v += dpp_mov<0x140>(v); // row_mirror
  if (L >= 32) v += __shfl_xor(v, 16);
  if (L >= 64) v += __shfl_xor(v, 32);
  return v;
}

}  // namespace lsh
