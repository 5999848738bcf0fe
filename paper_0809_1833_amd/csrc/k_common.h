// Wave64 / workgroup reductions used by the decoder's kernels (gfx950).
//
// All reductions combine values in a fixed pattern (DPP steps inside each
// 16-lane row, the rows in lane order, then the per-wave results in wave
// order), so a given launch shape always produces bit-identical results.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mp_internal.h"

namespace mp {

constexpr int kWave = 64;
typedef float v4f __attribute__((ext_vector_type(4)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));

// ---- cross-lane reductions ---------------------------------------------------
//
// Inside each row of 16 lanes the reductions use DPP lane moves, which run on
// the vector ALU instead of the LDS crossbar.
//
// Sums of floats (the inner products) keep every lane's result identical, as
// the per-lane candidate lists that follow require: quad_perm [1,0,3,2] and
// [2,3,0,1], row_mirror (lane i <-> 15-i) and row_half_mirror (i <-> 7-i)
// are all symmetric exchanges, so after the four steps all 16 lanes of a row
// hold the same row sum (addition is commutative), and two xor shuffles
// across rows (16, then 32) finish it the same way.
//
// The 64-bit maximum and the FP64 sum return a wave-uniform value: after
// quad_perm [1,0,3,2], [2,3,0,1], row_ror:4 and row_ror:8, lane 16k holds a
// fixed combination of row k's values, and lanes 0, 16, 32 and 48 are then
// read and combined in a fixed order.
//
// Every pattern depends only on the lane, so results are bit-reproducible.
// Callers run these with every lane of the wave active.
constexpr int kDppQuadSwap1 = 0xB1;      // quad_perm [1,0,3,2]
constexpr int kDppQuadSwap2 = 0x4E;      // quad_perm [2,3,0,1]
constexpr int kDppRowRor4 = 0x124;       // row_ror:4
constexpr int kDppRowRor8 = 0x128;       // row_ror:8
constexpr int kDppRowMirror = 0x140;     // row_mirror
constexpr int kDppRowHalfMirror = 0x141; // row_half_mirror
constexpr int kDppRowShl4 = 0x104;       // row_shl:4 (lane i reads lane i+4 of its row)
constexpr int kDppRowShr4 = 0x114;       // row_shr:4 (lane i reads lane i-4 of its row)

template <int CTRL>
__device__ inline uint32_t dpp_u32(uint32_t v) {
  return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(
      static_cast<int>(v), static_cast<int>(v), CTRL, 0xF, 0xF, false));
}

template <int CTRL>
__device__ inline float dpp_f32(float v) {
  return __builtin_bit_cast(float, dpp_u32<CTRL>(__builtin_bit_cast(uint32_t, v)));
}

template <int CTRL>
__device__ inline uint64_t dpp_u64(uint64_t v) {
  const uint32_t lo = dpp_u32<CTRL>(static_cast<uint32_t>(v));
  const uint32_t hi = dpp_u32<CTRL>(static_cast<uint32_t>(v >> 32));
  return (static_cast<uint64_t>(hi) << 32) | lo;
}

template <int CTRL>
__device__ inline double dpp_f64(double v) {
  return __builtin_bit_cast(double, dpp_u64<CTRL>(__builtin_bit_cast(uint64_t, v)));
}

__device__ inline uint64_t lane_u64(uint64_t v, int l) {
  const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), l));
  const uint32_t hi =
      static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v >> 32), l));
  return (static_cast<uint64_t>(hi) << 32) | lo;
}

__device__ inline double lane_f64(double v, int l) {
  return __builtin_bit_cast(double, lane_u64(__builtin_bit_cast(uint64_t, v), l));
}

__device__ inline uint64_t umax64(uint64_t a, uint64_t b) { return a > b ? a : b; }

__device__ inline float wave_sum(float v) {
  v += dpp_f32<kDppQuadSwap1>(v);
  v += dpp_f32<kDppQuadSwap2>(v);
  v += dpp_f32<kDppRowMirror>(v);
  v += dpp_f32<kDppRowHalfMirror>(v);
  v += __shfl_xor(v, 16, kWave);
  v += __shfl_xor(v, 32, kWave);
  return v;
}

__device__ inline double wave_sum(double v) {
  v += dpp_f64<kDppQuadSwap1>(v);
  v += dpp_f64<kDppQuadSwap2>(v);
  v += dpp_f64<kDppRowRor4>(v);
  v += dpp_f64<kDppRowRor8>(v);
  return (lane_f64(v, 0) + lane_f64(v, 16)) + (lane_f64(v, 32) + lane_f64(v, 48));
}

__device__ inline uint64_t wave_max(uint64_t v) {
  v = umax64(v, dpp_u64<kDppQuadSwap1>(v));
  v = umax64(v, dpp_u64<kDppQuadSwap2>(v));
  v = umax64(v, dpp_u64<kDppRowRor4>(v));
  v = umax64(v, dpp_u64<kDppRowRor8>(v));
  return umax64(umax64(lane_u64(v, 0), lane_u64(v, 16)), umax64(lane_u64(v, 32), lane_u64(v, 48)));
}

// Workgroup-wide sum of a double; every thread receives the result.
// `red` must hold NT/64 doubles of LDS.
template <int NT>
__device__ inline double block_sum(double v, double* red) {
  constexpr int NW = NT / kWave;
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  v = wave_sum(v);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = lane < NW ? red[lane] : 0.0;
  s = wave_sum(s);
  __syncthreads();  // red may be reused by the caller
  return s;
}

// Workgroup-wide max of a 64-bit key; every thread receives the result.
template <int NT>
__device__ inline uint64_t block_max(uint64_t v, uint64_t* red) {
  constexpr int NW = NT / kWave;
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  v = wave_max(v);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  uint64_t s = lane < NW ? red[lane] : 0ull;
  s = wave_max(s);
  __syncthreads();
  return s;
}

// ---- FP32 inner product of one column with the LDS copy of r ----------------
//
// The inner product is defined as two per-lane chains over the two halves of
// the column's float4s (ld4 is even: ld is a multiple of 64): lane l sums
// float4s l, l+64, ... below h0 = ld4/2 into one FP32 accumulator and
// h0+l, h0+l+64, ... into another, each in increasing order with FMAs; the
// two are added per lane and the wave sums the lanes.  A single wave runs both
// chains in lockstep; the re-scoring in the reduced-precision kernel gives
// each chain to its own wave and combines them per lane through LDS, with the
// same result bit for bit.

// U loads of 16 bytes in flight per lane, then U x 4 FMAs against the LDS
// copy of r; advances i by 64 * U float4s.  Streaming passes load with the
// non-temporal hint; STREAM = false keeps the lines cached (a column read
// again soon after).
template <int U, bool STREAM = true>
__device__ inline void dot_block(const v4f* __restrict__ p, const v4f* __restrict__ r_lds,
                                 int& i, float& acc) {
  v4f a[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if constexpr (STREAM) a[u] = __builtin_nontemporal_load(p + i + kWave * u);
    else a[u] = p[i + kWave * u];
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const v4f b = r_lds[i + kWave * u];
    acc = __builtin_fmaf(a[u].x, b.x, acc);
    acc = __builtin_fmaf(a[u].y, b.y, acc);
    acc = __builtin_fmaf(a[u].z, b.z, acc);
    acc = __builtin_fmaf(a[u].w, b.w, acc);
  }
  i += kWave * U;
}

// Both chains at once: U loads from each half (2U in flight per lane).
template <int U, bool STREAM = true>
__device__ inline void dot_block2(const v4f* __restrict__ p, const v4f* __restrict__ r_lds,
                                  int h0, int& i, float& acc_a, float& acc_b) {
  v4f a[U], b[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if constexpr (STREAM) {
      a[u] = __builtin_nontemporal_load(p + i + kWave * u);
      b[u] = __builtin_nontemporal_load(p + h0 + i + kWave * u);
    } else {
      a[u] = p[i + kWave * u];
      b[u] = p[h0 + i + kWave * u];
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const v4f ra = r_lds[i + kWave * u];
    acc_a = __builtin_fmaf(a[u].x, ra.x, acc_a);
    acc_a = __builtin_fmaf(a[u].y, ra.y, acc_a);
    acc_a = __builtin_fmaf(a[u].z, ra.z, acc_a);
    acc_a = __builtin_fmaf(a[u].w, ra.w, acc_a);
    const v4f rb = r_lds[h0 + i + kWave * u];
    acc_b = __builtin_fmaf(b[u].x, rb.x, acc_b);
    acc_b = __builtin_fmaf(b[u].y, rb.y, acc_b);
    acc_b = __builtin_fmaf(b[u].z, rb.z, acc_b);
    acc_b = __builtin_fmaf(b[u].w, rb.w, acc_b);
  }
  i += kWave * U;
}

// <r, psi_col> for one column by one wave: both chains in blocks of 8 loads
// each while they fit, then at most one block each of 4, 2 and 1 (so short
// columns still have several loads in flight), then the lane sum.  STREAM =
// false keeps the column's lines cached (a vector read again soon).
template <bool STREAM = true>
__device__ inline float dot_column_f32(const v4f* __restrict__ p, const v4f* __restrict__ r_lds,
                                       int ld4, int lane) {
  const int h0 = ld4 / 2;
  float acc_a = 0.0f, acc_b = 0.0f;
  int i = lane;
  while (i + kWave * 7 < h0) dot_block2<8, STREAM>(p, r_lds, h0, i, acc_a, acc_b);
  if (i + kWave * 3 < h0) dot_block2<4, STREAM>(p, r_lds, h0, i, acc_a, acc_b);
  if (i + kWave * 1 < h0) dot_block2<2, STREAM>(p, r_lds, h0, i, acc_a, acc_b);
  if (i < h0) dot_block2<1, STREAM>(p, r_lds, h0, i, acc_a, acc_b);
  return wave_sum(acc_a + acc_b);
}

// One chain of the inner product (float4s base+l, base+l+64, ... below
// base+len) as this lane's partial sum, without the lane sum.  Used for
// re-scoring, whose winning column is read again by the update, so its lines
// stay cached.
__device__ inline float dot_chain_f32(const v4f* __restrict__ p, const v4f* __restrict__ r_lds,
                                      int base, int len, int lane) {
  p += base;
  r_lds += base;
  float acc = 0.0f;
  int i = lane;
  while (i + kWave * 15 < len) dot_block<16, false>(p, r_lds, i, acc);
  if (i + kWave * 7 < len) dot_block<8, false>(p, r_lds, i, acc);
  if (i + kWave * 3 < len) dot_block<4, false>(p, r_lds, i, acc);
  if (i + kWave * 1 < len) dot_block<2, false>(p, r_lds, i, acc);
  if (i < len) dot_block<1, false>(p, r_lds, i, acc);
  return acc;
}

// ---- hand-off from all workgroups of a launch to the last one (OMP) ---------
//
// Each workgroup publishes K keys into its own K slots of `keys` and counts
// itself in; publish_arrive returns true (in every thread) only in the
// workgroup that arrives last.
//
// The key slots and the arrival counter are only ever touched with atomic
// read-modify-write operations at device scope.  Each one is performed at
// the device's point of coherence for atomics and returns only once
// performed, and every RMW returns the latest value of its word.  A
// workgroup swaps its keys into its slots, waits for those swaps to return,
// then increments the counter; the workgroup whose increment returns grid-1
// issues its reads (take_slot: a swap with zero, which also clears the slot
// for the next launch) after that, so they return the keys stored in this
// launch.  Plain or relaxed loads are never used for these words: a relaxed
// load is not ordered after other workgroups' RMWs and could return an older
// value.  No cache write-back or invalidate is needed; everything else the
// last workgroup reads was written by earlier launches.
//
// `mine` must hold the workgroup's j-th key in lane j of wave 0, j < K.
template <int K>
__device__ inline bool publish_arrive(uint64_t mine, uint64_t* keys, DevState* st) {
  static_assert(K >= 1 && K <= kWave, "K keys per workgroup");
  __shared__ int s_last;
  if (threadIdx.x < kWave) {
    const int lane = threadIdx.x;
    uint64_t old = 0;
    if (lane < K)
      old = __hip_atomic_exchange(keys + static_cast<size_t>(blockIdx.x) * K + lane, mine,
                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // Keys never have bit 63 set, so inc is 1; computing it from every lane's
    // returned value makes the increment wait for all K swaps to be performed.
    const unsigned long long high = __ballot((old >> 63) != 0);
    if (lane == 0) {
      const unsigned inc = 1u + (high != 0ull ? 1u : 0u);
      const unsigned prev =
          __hip_atomic_fetch_add(&st->arrive, inc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const int last = prev == gridDim.x - 1;
      if (last)
        (void)__hip_atomic_exchange(&st->arrive, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_last = last;
    }
  }
  __syncthreads();
  return s_last != 0;
}

// Read (and clear) one published key slot; only in the last workgroup.
__device__ inline uint64_t take_slot(uint64_t* slot) {
  return __hip_atomic_exchange(slot, uint64_t{0}, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---- balanced column shares of the carried FP32 pass ---------------------
//
// Launch k takes its group shares from launch k-1's shares and pass
// durations (both written before the kernel boundary): each group's rate
// (columns per tick per workgroup), the count that would make every group
// finish together, then a step of kBalStep from the old count toward it,
// clamped to [cpw/2, 3 cpw/2] and rounded down, with one column added to
// groups in turn until the shares cover all m columns.  Every workgroup computes the same
// integers from the same inputs.  Workgroup b = 8q + g takes
// [q * S + sum_{h<g} s_h, + s_g) clipped to m, S = sum_h s_h, so the ranges
// tile [0, m) in blockIdx order.  Launch 0, grids that are not a multiple
// of 8 and workgroups of fewer than four columns per wave use cpw each.
//
// dur_prev: this thread's workgroup-indexed duration of launch k-1 (thread
// t < grid), sh_prev: share[par ^ 1][t] (t < 8); both requested by the
// caller with its other loads.  Every thread calls; there are barriers.
constexpr float kBalStep = 0.5f;

template <int NT>
__device__ void balanced_range(BalState* __restrict__ bal, int par, bool adapt, int grid,
                               int64_t m, int cpw, unsigned dur_prev, int sh_prev,
                               int64_t& col0, int64_t& col1) {
  static_assert(NT >= kBalMaxGrid, "one duration per thread");
  __shared__ unsigned s_dur[kBalMaxGrid];
  __shared__ float s_rate[kBalGroups];
  __shared__ int s_sh[kBalGroups];
  const int t = threadIdx.x;
  const int ngr = grid / kBalGroups;  // workgroups per group
  adapt = adapt && grid % kBalGroups == 0 && cpw >= 64 && grid <= kBalMaxGrid;
  if (adapt) {
    if (t < grid) s_dur[t] = dur_prev;  // grid <= kBalMaxGrid <= NT
    __syncthreads();
    if (t < kBalGroups) {
      float sum = 0.0f;
      for (int q = 0; q < ngr; ++q) sum += static_cast<float>(s_dur[q * kBalGroups + t]);
      const float mean = sum / static_cast<float>(ngr);
      s_rate[t] = sh_prev > 0 && mean > 0.0f ? static_cast<float>(sh_prev) / mean : 0.0f;
      s_sh[t] = sh_prev;
    }
    __syncthreads();
    if (t == 0) {
      bool ok = true;
      float tot = 0.0f;
      for (int g = 0; g < kBalGroups; ++g) {
        ok = ok && s_rate[g] > 0.0f;
        tot += s_rate[g];
      }
      int sh[kBalGroups];
      int64_t cover = 0;
      for (int g = 0; g < kBalGroups; ++g) {
        float target = ok ? static_cast<float>(m) / static_cast<float>(ngr) * (s_rate[g] / tot)
                          : static_cast<float>(cpw);
        float v = ok ? (1.0f - kBalStep) * static_cast<float>(s_sh[g]) + kBalStep * target
                     : target;
        v = v < 0.5f * cpw ? 0.5f * cpw : (v > 1.5f * cpw ? 1.5f * cpw : v);
        sh[g] = static_cast<int>(v);
        cover += static_cast<int64_t>(ngr) * sh[g];
      }
      for (int g = 0; cover < m; g = (g + 1) % kBalGroups) {
        ++sh[g];
        cover += ngr;
      }
      for (int g = 0; g < kBalGroups; ++g) s_sh[g] = sh[g];
    }
    __syncthreads();
  } else if (t < kBalGroups) {
    s_sh[t] = cpw;
  }
  if (!adapt) __syncthreads();
  int S = 0, before = 0;
  const int g = static_cast<int>(blockIdx.x) % kBalGroups;
  for (int h = 0; h < kBalGroups; ++h) {
    S += s_sh[h];
    before += h < g ? s_sh[h] : 0;
  }
  const int64_t q = static_cast<int64_t>(blockIdx.x) / kBalGroups;
  col0 = adapt ? q * S + before : static_cast<int64_t>(blockIdx.x) * cpw;
  col1 = col0 + (adapt ? s_sh[g] : cpw);
  if (col0 > m) col0 = m;
  if (col1 > m) col1 = m;
  if (blockIdx.x == 0 && t < kBalGroups) bal->share[par][t] = adapt ? s_sh[t] : cpw;
}

// The workgroup's pass duration for the next launch (thread 0).
__device__ inline void record_pass_time(BalState* __restrict__ bal, int par,
                                        unsigned long long t_begin) {
  if (threadIdx.x == 0 && blockIdx.x < kBalMaxGrid)
    bal->dur[par][blockIdx.x] = static_cast<unsigned>(wall_clock64() - t_begin);
}

// ---- steps carried into the next launch ------------------------------------
//
// The FP32 and reduced-precision forms finish step k at the start of launch
// k+1 (k counted from 1): every workgroup finds the same winner (idx, c) and
// applies the step to its own LDS copy of r, so no workgroup hands anything
// to another inside a launch; the kernel boundary orders the published keys.

// The winner cannot be applied (an index outside the dictionary, which no
// published key holds, or c = 0: no atom correlates with r): workgroup 0
// records the stop.  Same value in every thread of every workgroup.
__device__ inline bool carried_winner_stops(int idx, float c, int64_t m,
                                            DevState* __restrict__ st) {
  const bool bad = idx < 0 || idx >= m;
  if (!bad && c != 0.0f) return false;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->reason = bad ? kStopInternal : MP_STOP_STALLED;
    st->done = 1;
  }
  return true;
}

// Rows 4i..4i+3 of a residual into a trace entry (rows below n only).
__device__ inline void trace_rows4(float* __restrict__ dst, int i, int64_t n, const v4f& o) {
  const int64_t row = 4 * static_cast<int64_t>(i);
  if (row < n) dst[row] = o.x;
  if (row + 1 < n) dst[row + 1] = o.y;
  if (row + 2 < n) dst[row + 2] = o.z;
  if (row + 3 < n) dst[row + 3] = o.w;
}

// Step k applied in every workgroup: r -= c psi_idx with the FP32 column (one
// FMA per element, padding rows stay +0) on the LDS copy and ||r||^2 in FP64
// (per-thread sums over its float4s in order, then block_sum: the same value
// in every workgroup); workgroup 0 also stores r in r_out, adds c to x~_idx
// (eq. 10) and writes the trace entry (with the residual's n rows when the
// trace asks for them) and the state (t = k, eq. 12, the stop test, `half` =
// the half of the residual buffer r_out is).  Returns true, in every thread
// of every workgroup, when the run stops after step k.
template <int NT>
__device__ bool carried_update(int idx, float c, const float* __restrict__ psi32, int64_t ld,
                               int64_t n, v4f* __restrict__ r_lds, v4f* __restrict__ r_out,
                               float* __restrict__ x, DevState* __restrict__ st,
                               const mp_trace& tr, long long k, long long max_iters, double thr,
                               int half, double* dred) {
  constexpr int P = 16384 / 4 / NT > 0 ? 16384 / 4 / NT : 1;  // ld <= 16384
  const int ld4 = static_cast<int>(ld / 4);
  const v4f* col = reinterpret_cast<const v4f*>(psi32 + static_cast<int64_t>(idx) * ld);
  v4f a[P];
#pragma unroll
  for (int u = 0; u < P; ++u) {
    const int i = threadIdx.x + u * NT;
    a[u] = col[i < ld4 ? i : ld4 - 1];
  }
  float* rt = nullptr;  // this step's residual trace entry (workgroup 0 only)
  if (blockIdx.x == 0 && tr.r && k - 1 < tr.cap) rt = tr.r + (k - 1) * tr.ldr;
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < P; ++u) {
    const int i = threadIdx.x + u * NT;
    if (i < ld4) {
      const v4f rv = r_lds[i];
      v4f o;
      o.x = __builtin_fmaf(-c, a[u].x, rv.x);
      o.y = __builtin_fmaf(-c, a[u].y, rv.y);
      o.z = __builtin_fmaf(-c, a[u].z, rv.z);
      o.w = __builtin_fmaf(-c, a[u].w, rv.w);
      r_lds[i] = o;
      if (blockIdx.x == 0) r_out[i] = o;
      if (rt) trace_rows4(rt, i, n, o);
      s += static_cast<double>(o.x) * o.x + static_cast<double>(o.y) * o.y +
           (static_cast<double>(o.z) * o.z + static_cast<double>(o.w) * o.w);
    }
  }
  const double rr = block_sum<NT>(s, dred);  // its barriers also order the r_lds writes
  const bool stop = !(rr > thr) || k >= max_iters;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    x[idx] += c;
    const long long t = k - 1;
    if (t < tr.cap) {
      if (tr.idx) tr.idx[t] = idx;
      if (tr.coef) tr.coef[t] = c;
      if (tr.rr) tr.rr[t] = rr;
    }
    st->t = k;
    st->rr = rr;
    st->r_sel = half;
    if (!(rr > thr)) {
      st->reason = MP_STOP_CONVERGED;
      st->done = 1;
    } else if (k >= max_iters) {
      st->reason = MP_STOP_MAX_ITERS;
      st->done = 1;
    }
  }
  return stop;
}

}  // namespace mp
