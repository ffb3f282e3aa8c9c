// Wavefront-level sums on CDNA (64 lanes) through DPP lane permutes, which stay
// in the vector ALU (a shuffle through LDS costs a round trip per step).
#pragma once

#include <hip/hip_runtime.h>

namespace seqx {

// one DPP move of both halves of a double (lanes outside ROWS read 0)
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ double dpp_move(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b), CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), CTRL, ROWS, 0xf, false);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

// sum over the 64 lanes in a fixed order, returned in every lane: pairs,
// quads, half rows and rows by DPP permutes, then rows 0+1 and (0+1)+2+3 by
// the row broadcasts of lanes 15 and 31; the total ends in lane 63
__device__ __forceinline__ double wave_sum64(double s) {
  s += dpp_move<0xb1>(s);        // quad_perm [1,0,3,2]
  s += dpp_move<0x4e>(s);        // quad_perm [2,3,0,1]
  s += dpp_move<0x141>(s);       // row_half_mirror
  s += dpp_move<0x140>(s);       // row_mirror
  s += dpp_move<0x142, 0xa>(s);  // row_bcast:15 into rows 1, 3
  s += dpp_move<0x143, 0xc>(s);  // row_bcast:31 into rows 2, 3
  const long long b = __double_as_longlong(s);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(b), 63);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), 63);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

}  // namespace seqx
