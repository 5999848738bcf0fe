// Shared pieces of the reduced-precision and multi-candidate kernels:
// BF16 rounding, reduced-precision inner products against an FP32 residual
// in LDS, and top-8 lists of packed candidate keys.
#pragma once

#include "k_common.h"

namespace mp {

typedef float v2f __attribute__((ext_vector_type(2)));
constexpr int kTopK = 8;

// FP32 -> BF16 bit pattern, round to nearest even (finite inputs).
__device__ inline uint16_t bf16_rne(float v) {
  uint32_t u = __builtin_bit_cast(uint32_t, v);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}

// ---------------------------------------------------------------------------
// Reduced-precision inner products.  S = bytes per element (2: BF16, 1: FP8);
// one 16-byte load holds E = 16 / S elements, matched by E / 4 float4s of r.

template <int S>
__device__ inline void lp_fma(v4u q, const v4f* __restrict__ rv, float& acc) {
  if constexpr (S == 2) {
    const v4f b0 = rv[0], b1 = rv[1];
    acc = __builtin_fmaf(__builtin_bit_cast(float, q.x << 16), b0.x, acc);
    acc = __builtin_fmaf(__builtin_bit_cast(float, q.x & 0xFFFF0000u), b0.y, acc);
    acc = __builtin_fmaf(__builtin_bit_cast(float, q.y << 16), b0.z, acc);
    acc = __builtin_fmaf(__builtin_bit_cast(float, q.y & 0xFFFF0000u), b0.w, acc);
    acc = __builtin_fmaf(__builtin_bit_cast(float, q.z << 16), b1.x, acc);
    acc = __builtin_fmaf(__builtin_bit_cast(float, q.z & 0xFFFF0000u), b1.y, acc);
    acc = __builtin_fmaf(__builtin_bit_cast(float, q.w << 16), b1.z, acc);
    acc = __builtin_fmaf(__builtin_bit_cast(float, q.w & 0xFFFF0000u), b1.w, acc);
  } else {
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const v4f b = rv[w];
      const unsigned word = q[w];
      // gfx950 decodes OCP e4m3fn exactly: bytes 0,1 then bytes 2,3
      const v2f lo = __builtin_amdgcn_cvt_pk_f32_fp8(static_cast<int>(word), false);
      const v2f hi = __builtin_amdgcn_cvt_pk_f32_fp8(static_cast<int>(word), true);
      acc = __builtin_fmaf(lo.x, b.x, acc);
      acc = __builtin_fmaf(lo.y, b.y, acc);
      acc = __builtin_fmaf(hi.x, b.z, acc);
      acc = __builtin_fmaf(hi.y, b.w, acc);
    }
  }
}

template <int S, int U>
__device__ inline void lp_block(const v4u* __restrict__ p, const v4f* __restrict__ r_lds,
                                int& i, float& acc) {
  constexpr int R = 16 / S / 4;  // float4s of r per 16-byte load
  v4u a[U];
#pragma unroll
  for (int u = 0; u < U; ++u) a[u] = __builtin_nontemporal_load(p + i + kWave * u);
#pragma unroll
  for (int u = 0; u < U; ++u) lp_fma<S>(a[u], r_lds + (i + kWave * u) * R, acc);
  i += kWave * U;
}

// Reduced-precision <r, psi_col> (before the FP8 scale) by one wave; nq
// 16-byte chunks per column.
template <int S>
__device__ inline float dot_column_lp(const v4u* __restrict__ p, const v4f* __restrict__ r_lds,
                                      int nq, int lane) {
  float acc = 0.0f;
  int i = lane;
  while (i + kWave * 7 < nq) lp_block<S, 8>(p, r_lds, i, acc);
  if (i + kWave * 3 < nq) lp_block<S, 4>(p, r_lds, i, acc);
  if (i + kWave * 1 < nq) lp_block<S, 2>(p, r_lds, i, acc);
  if (i < nq) lp_block<S, 1>(p, r_lds, i, acc);
  return wave_sum(acc);
}

// CC columns at once by one wave (CC x U loads in flight per lane); each
// column's chunks are accumulated in the same order as dot_column_lp, so the
// results are identical.
template <int S, int U, int CC>
__device__ inline void lp_block_cols(const v4u* const (&p)[CC], const v4f* __restrict__ r_lds,
                                     int& i, float (&acc)[CC]) {
  constexpr int R = 16 / S / 4;
  v4u a[CC][U];
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int c = 0; c < CC; ++c) a[c][u] = __builtin_nontemporal_load(p[c] + i + kWave * u);
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int c = 0; c < CC; ++c) lp_fma<S>(a[c][u], r_lds + (i + kWave * u) * R, acc[c]);
  i += kWave * U;
}

template <int S, int CC>
__device__ inline void dot_columns_lp(const v4u* const (&p)[CC], const v4f* __restrict__ r_lds,
                                      int nq, int lane, float (&out)[CC]) {
  float acc[CC];
#pragma unroll
  for (int c = 0; c < CC; ++c) acc[c] = 0.0f;
  int i = lane;
  while (i + kWave * 7 < nq) lp_block_cols<S, 8, CC>(p, r_lds, i, acc);
  if (i + kWave * 3 < nq) lp_block_cols<S, 4, CC>(p, r_lds, i, acc);
  if (i + kWave * 1 < nq) lp_block_cols<S, 2, CC>(p, r_lds, i, acc);
  if (i < nq) lp_block_cols<S, 1, CC>(p, r_lds, i, acc);
#pragma unroll
  for (int c = 0; c < CC; ++c) out[c] = wave_sum(acc[c]);
}

// ---------------------------------------------------------------------------
// Top-8 lists of packed keys (larger key = larger |c|, then smaller index;
// 0 = empty).

// Insert into a sorted (descending) list; the smallest entry falls out.
__device__ inline void top8_insert(uint64_t (&L)[kTopK], uint64_t key) {
  if (key <= L[kTopK - 1]) return;
#pragma unroll
  for (int j = 0; j < kTopK; ++j) {
    if (key > L[j]) {
      const uint64_t t = L[j];
      L[j] = key;
      key = t;
    }
  }
}

// ---- sorting networks on keys held in one thread's registers ----------------

// Compare-exchange for descending order: a keeps the larger key.
__device__ inline void cx_keys(uint64_t& a, uint64_t& b) {
  const uint64_t hi = a > b ? a : b;
  b = a > b ? b : a;
  a = hi;
}

// Sorts 8 keys in descending order: a 19 compare-exchange network (checked
// on all 256 inputs of 0s and 1s, which suffices for a sorting network).
__device__ inline void sort8_keys(uint64_t (&v)[8]) {
  cx_keys(v[0], v[2]); cx_keys(v[1], v[3]); cx_keys(v[4], v[6]); cx_keys(v[5], v[7]);
  cx_keys(v[0], v[4]); cx_keys(v[1], v[5]); cx_keys(v[2], v[6]); cx_keys(v[3], v[7]);
  cx_keys(v[0], v[1]); cx_keys(v[2], v[3]); cx_keys(v[4], v[5]); cx_keys(v[6], v[7]);
  cx_keys(v[2], v[4]); cx_keys(v[3], v[5]);
  cx_keys(v[1], v[4]); cx_keys(v[3], v[6]);
  cx_keys(v[1], v[2]); cx_keys(v[3], v[4]); cx_keys(v[5], v[6]);
}

// a <- the 8 largest of two descending lists a and b, descending: the
// element-wise maximum of a and reversed b is bitonic and holds them; the
// bitonic merge (distances 4, 2, 1) sorts it.
__device__ inline void merge8_keys(uint64_t (&a)[8], const uint64_t (&b)[8]) {
#pragma unroll
  for (int i = 0; i < 8; ++i) a[i] = a[i] > b[7 - i] ? a[i] : b[7 - i];
  cx_keys(a[0], a[4]); cx_keys(a[1], a[5]); cx_keys(a[2], a[6]); cx_keys(a[3], a[7]);
  cx_keys(a[0], a[2]); cx_keys(a[1], a[3]); cx_keys(a[4], a[6]); cx_keys(a[5], a[7]);
  cx_keys(a[0], a[1]); cx_keys(a[2], a[3]); cx_keys(a[4], a[5]); cx_keys(a[6], a[7]);
}

// ---- bitonic merge of sorted 8-key lists across the lanes of a wave ----------

// Lane i receives lane (i ^ 4)'s key (groups of 8 lanes inside a row of 16).
__device__ inline uint64_t xor4_u64(uint64_t v, int lane) {
  const uint64_t up = dpp_u64<kDppRowShl4>(v);
  const uint64_t dn = dpp_u64<kDppRowShr4>(v);
  return (lane & 4) ? dn : up;
}

// Compare-exchange for descending order: the lower lane of a pair keeps the
// larger key.
__device__ inline uint64_t cx_desc(uint64_t v, uint64_t partner, bool upper) {
  return upper ? (v < partner ? v : partner) : (v > partner ? v : partner);
}

// Sorts, descending, the bitonic sequence of 8 keys each group of 8 lanes
// holds (compare-exchange at distances 4, 2, 1).
__device__ inline uint64_t bitonic_sort8(uint64_t v, int lane) {
  v = cx_desc(v, xor4_u64(v, lane), (lane & 4) != 0);
  v = cx_desc(v, dpp_u64<kDppQuadSwap2>(v), (lane & 2) != 0);
  v = cx_desc(v, dpp_u64<kDppQuadSwap1>(v), (lane & 1) != 0);
  return v;
}

__device__ inline uint64_t shfl_u64(uint64_t v, int src) {
  return __shfl(static_cast<unsigned long long>(v), src, kWave);
}

// The 8 largest keys of 16 lists of 8, each sorted in descending order: list
// g < 8 sits in lanes 8g..8g+7 of `a` (its rank-j key in lane 8g+j), list
// 8+g likewise in `b`.  The element-wise maximum of one sorted list and the
// reverse of another is a bitonic sequence holding the 8 largest keys of
// both, so four such merges (partner list reversed by row_half_mirror, then
// row_mirror, then lane ^ 23 and lane ^ 39) each followed by bitonic_sort8
// leave the 8 largest of all 128 keys, sorted, in every group of 8 lanes;
// lane j < 8 returns the j-th largest.  0 (an empty entry) sorts last.
__device__ inline uint64_t top8_of_lists16(uint64_t a, uint64_t b, int lane) {
  uint64_t v = umax64(a, dpp_u64<kDppRowHalfMirror>(b));
  v = bitonic_sort8(v, lane);
  v = umax64(v, dpp_u64<kDppRowMirror>(v));
  v = bitonic_sort8(v, lane);
  v = umax64(v, shfl_u64(v, lane ^ 23));
  v = bitonic_sort8(v, lane);
  v = umax64(v, shfl_u64(v, lane ^ 39));
  return bitonic_sort8(v, lane);
}

// The 8 largest of two descending lists held in every group of 8 lanes (rank
// j in lane 8g + j), sorted the same way.
__device__ inline uint64_t merge_lane_lists8(uint64_t a, uint64_t b, int lane) {
  return bitonic_sort8(umax64(a, dpp_u64<kDppRowHalfMirror>(b)), lane);
}

}  // namespace mp
