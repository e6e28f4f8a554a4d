// Wave-level helpers shared by the HIP kernels (device code only).
#pragma once
#include <hip/hip_runtime.h>

namespace ttn {

// v + (v moved by the DPP pattern CTRL), the two 32-bit halves moved separately
template <int CTRL>
__device__ __forceinline__ double dpp_add(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return v + __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double lane_value(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Wave sum without the LDS crossbar: within each row of 16 lanes by DPP
// (rotate by 8 and by 4, then swap pairs of 2 and of 1), then the four row sums
// read from lanes 0, 16, 32, 48.  The result is wave-uniform.
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v = dpp_add<0x128>(v);  // row_ror:8
  v = dpp_add<0x124>(v);  // row_ror:4
  v = dpp_add<0x4E>(v);   // quad_perm [2,3,0,1]
  v = dpp_add<0xB1>(v);   // quad_perm [1,0,3,2]
  return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

}  // namespace ttn
