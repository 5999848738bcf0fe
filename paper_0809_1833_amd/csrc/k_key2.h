// A candidate of the FP64 argmax as a pair of 64-bit words, so that the exact
// FP64 coefficient survives the reduction: the |c| bits (a non-negative
// double orders like its bit pattern), then (0x7FFFFFFF - index) and the
// sign.  The pair order is "larger |c|, then smaller index" (eq. 16).
#pragma once

#include "k_common.h"

namespace mp {

struct Key2 {
  uint64_t hi;  // |c| bits, sign cleared (NaN mapped to 0)
  uint64_t lo;  // (0x7FFFFFFF - index) << 1 | sign of c; 0 = empty
};

__device__ inline Key2 make_key2(double c, int idx) {
  const uint64_t u = __builtin_bit_cast(uint64_t, c);
  uint64_t ab = u & 0x7FFFFFFFFFFFFFFFull;
  if (ab > 0x7FF0000000000000ull) ab = 0;
  return Key2{ab, (static_cast<uint64_t>(0x7FFFFFFFu - static_cast<uint32_t>(idx)) << 1) |
                      (u >> 63)};
}
__device__ inline int key2_index(const Key2& k) {
  return static_cast<int>(0x7FFFFFFFu - (static_cast<uint32_t>(k.lo) >> 1));
}
__device__ inline double key2_value(const Key2& k) {
  return __builtin_bit_cast(double, k.hi | ((k.lo & 1ull) << 63));
}
__device__ inline bool key2_greater(const Key2& a, const Key2& b) {
  return a.hi > b.hi || (a.hi == b.hi && a.lo > b.lo);
}
__device__ inline Key2 key2_max(const Key2& a, const Key2& b) {
  return key2_greater(b, a) ? b : a;
}

template <int CTRL>
__device__ inline Key2 dpp_key2(const Key2& k) {
  return Key2{dpp_u64<CTRL>(k.hi), dpp_u64<CTRL>(k.lo)};
}
__device__ inline Key2 lane_key2(const Key2& k, int l) {
  return Key2{lane_u64(k.hi, l), lane_u64(k.lo, l)};
}

// Wave-uniform maximum pair (the DPP pattern of wave_max).
__device__ inline Key2 wave_max_key2(Key2 k) {
  k = key2_max(k, dpp_key2<kDppQuadSwap1>(k));
  k = key2_max(k, dpp_key2<kDppQuadSwap2>(k));
  k = key2_max(k, dpp_key2<kDppRowRor4>(k));
  k = key2_max(k, dpp_key2<kDppRowRor8>(k));
  return key2_max(key2_max(lane_key2(k, 0), lane_key2(k, 16)),
                  key2_max(lane_key2(k, 32), lane_key2(k, 48)));
}

// Workgroup-wide maximum pair; every thread receives it.  `red` holds NT/64
// pairs of LDS.
template <int NT>
__device__ inline Key2 block_max_key2(Key2 k, Key2* red) {
  constexpr int NW = NT / kWave;
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  k = wave_max_key2(k);
  if (lane == 0) red[wave] = k;
  __syncthreads();
  Key2 s = lane < NW ? red[lane] : Key2{0, 0};
  s = wave_max_key2(s);
  __syncthreads();
  return s;
}

}  // namespace mp
