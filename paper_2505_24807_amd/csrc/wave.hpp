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

// the value of x in lane src (src uniform across the wavefront)
__device__ __forceinline__ double lane_value(double x, int src) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(b), src);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), src);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

// the value of lane ^ M: DPP moves inside 16-lane rows for M = 1, 2 (quad
// permutes) and 8 (row rotation by 8), ds_swizzle in bit mode for M = 4, 16
// (within 32-lane halves), ds_bpermute for M = 32
template <int M>
__device__ __forceinline__ double xor_shuffle(double x) {
  if constexpr (M == 1) return dpp_move<0xb1>(x);   // quad_perm [1,0,3,2]
  if constexpr (M == 2) return dpp_move<0x4e>(x);   // quad_perm [2,3,0,1]
  if constexpr (M == 8) return dpp_move<0x128>(x);  // row_ror:8
  const long long b = __double_as_longlong(x);
  int lo = static_cast<int>(b), hi = static_cast<int>(b >> 32);
  if constexpr (M < 32) {
    constexpr int pattern = (M << 10) | 0x1f;  // and-mask 31, or-mask 0, xor-mask M
    lo = __builtin_amdgcn_ds_swizzle(lo, pattern);
    hi = __builtin_amdgcn_ds_swizzle(hi, pattern);
  } else {
    const int addr = ((threadIdx.x & 63) ^ 32) << 2;
    lo = __builtin_amdgcn_ds_bpermute(addr, lo);
    hi = __builtin_amdgcn_ds_bpermute(addr, hi);
  }
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

// one butterfly level: lanes paired by bit M keep H of their 2H values (the
// upper lane the upper half) and add the partner's copy of them
template <int M, int H>
__device__ __forceinline__ void butterfly_level(double* x) {
  const bool up = (threadIdx.x & M) != 0;
#pragma unroll
  for (int k = 0; k < H; ++k) {
    const double send = up ? x[k] : x[k + H];
    const double keep = up ? x[k + H] : x[k];
    x[k] = keep + xor_shuffle<M>(send);
  }
}

// sums of 8 values per lane over the 64 lanes, in a fixed order: returns in
// lane L the total of x[(L >> 3) & 7] (10 exchanges instead of 8 x 6; the
// last four are DPP moves, the 8-lane sums pairing lane i with 7 - i first)
__device__ __forceinline__ double wave_sum8x64(double (&x)[8]) {
  butterfly_level<32, 4>(x);
  butterfly_level<16, 2>(x);
  butterfly_level<8, 1>(x);
  double s = x[0];
  s += dpp_move<0x141>(s);  // row_half_mirror
  s += xor_shuffle<2>(s);
  s += xor_shuffle<1>(s);
  return s;
}

}  // namespace seqx
