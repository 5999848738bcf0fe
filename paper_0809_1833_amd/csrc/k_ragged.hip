// Many independent Matching Pursuit problems of uneven size in one launch.
//
// Every instance has its own dictionary and signal.  A persistent grid of
// workgroups takes items from an on-device work list (largest first, as the
// host ordered them) and runs one instance's whole Section 3 loop (eqs. 8-12)
// for each: the residual stays in LDS, the correlation pass streams the
// instance's dictionary with every wave taking CC columns at a time (short
// columns, of at most 32 16-byte elements, side by side in lane groups), and
// the argmax (smallest index on ties, eq. 16), the x~ and r updates and the FP64
// stopping test use only workgroup barriers.  An instance whose work would
// hold one workgroup far longer than the average item is cut by the host
// into `parts` consecutive items, one per column share: every part keeps the
// whole residual, streams its own columns and, each step, publishes its best
// candidates (FP32: one key; BF16: its 8 best) as self-tagged 64-bit words
// (32-bit tag = step + 1 over 32 bits of a key, relaxed device-scope
// atomics) and reads its siblings' words of the same step, so that every
// part takes the same winner and applies the same update with the same
// arithmetic (part 0 alone writes x~, the trace, r and the result).  Steps
// alternate between two halves of the instance's record slot: a part
// overwrites its words of step t only after reading every record of step
// t + 1, each published after its owner read every record of step t.  The
// slots are cleared before every decode.  Results do not depend on the
// split.  Every wait ends: the parts of an instance are consecutive in the
// list, so whenever the workgroups resident at once outnumber the parts of
// one instance, some complete group of parts is running; and a wait that
// polls `spin_limit` times in vain sets the queue's fail word and leaves the
// instance, after which its siblings' waits give up too.
//
// With BF16 storage each wave keeps the 8 best reduced-precision candidates
// of its columns; the workgroup merges them, re-scores up to 8 against the
// FP32 columns and takes the best re-scored one.
#include "k_common.h"
#include "k_lowp.h"
#include "mp_internal.h"

namespace mp {

// <r, psi_c> for CC columns at once by one wave (16-byte loads, 4 per column
// in flight per lane, then singles), FP32 accumulation, butterfly sums.
template <int CC>
__device__ inline void dot_cols_f32(const v4f* const (&p)[CC], const v4f* __restrict__ r_lds,
                                    int ld4, int lane, float (&acc)[CC]) {
#pragma unroll
  for (int c = 0; c < CC; ++c) acc[c] = 0.0f;
  int i = lane;
  for (; i + kWave * 3 < ld4; i += kWave * 4) {
    v4f a[CC][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int c = 0; c < CC; ++c) a[c][u] = __builtin_nontemporal_load(p[c] + i + kWave * u);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const v4f b = r_lds[i + kWave * u];
#pragma unroll
      for (int c = 0; c < CC; ++c) {
        acc[c] = __builtin_fmaf(a[c][u].x, b.x, acc[c]);
        acc[c] = __builtin_fmaf(a[c][u].y, b.y, acc[c]);
        acc[c] = __builtin_fmaf(a[c][u].z, b.z, acc[c]);
        acc[c] = __builtin_fmaf(a[c][u].w, b.w, acc[c]);
      }
    }
  }
  for (; i < ld4; i += kWave) {
    const v4f b = r_lds[i];
#pragma unroll
    for (int c = 0; c < CC; ++c) {
      const v4f a = __builtin_nontemporal_load(p[c] + i);
      acc[c] = __builtin_fmaf(a.x, b.x, acc[c]);
      acc[c] = __builtin_fmaf(a.y, b.y, acc[c]);
      acc[c] = __builtin_fmaf(a.z, b.z, acc[c]);
      acc[c] = __builtin_fmaf(a.w, b.w, acc[c]);
    }
  }
#pragma unroll
  for (int c = 0; c < CC; ++c) acc[c] = wave_sum(acc[c]);
}

// dot_columns_lp's sums (BF16 storage) with at most 8 16-byte loads in
// flight per lane in all: blocks of 8/CC per column, so that a 1024-thread
// workgroup's register share holds them.  A lane's sum runs over its
// elements i, i+64, i+128, ... in order whatever the blocking, so every sum
// is dot_columns_lp's bit for bit.
template <int CC>
__device__ inline void dot_cols_lp(const v4u* const (&p)[CC], const v4f* __restrict__ r_lds,
                                   int nq, int lane, float (&out)[CC]) {
  constexpr int U = 8 / CC;
  float acc[CC];
#pragma unroll
  for (int c = 0; c < CC; ++c) acc[c] = 0.0f;
  int i = lane;
  while (i + kWave * (U - 1) < nq) lp_block_cols<2, U, CC>(p, r_lds, i, acc);
  if constexpr (U >= 8)
    if (i + kWave * 3 < nq) lp_block_cols<2, 4, CC>(p, r_lds, i, acc);
  if constexpr (U >= 4)
    if (i + kWave * 1 < nq) lp_block_cols<2, 2, CC>(p, r_lds, i, acc);
  if constexpr (U >= 2)
    if (i < nq) lp_block_cols<2, 1, CC>(p, r_lds, i, acc);
#pragma unroll
  for (int c = 0; c < CC; ++c) out[c] = wave_sum(acc[c]);
}

// The correlation pass of one step over columns [cb, ce), CC columns at a
// time per wave.  FP32: returns the best key of this wave's columns.
template <int CC>
__device__ inline uint64_t f32_pass_wave(const float* __restrict__ psi32, int64_t ld, int ld4,
                                         const v4f* __restrict__ r_lds, int64_t cb, int64_t ce,
                                         int wave, int W, int lane) {
  uint64_t best = 0;
  for (int64_t c0 = cb + static_cast<int64_t>(wave) * CC; c0 < ce;
       c0 += static_cast<int64_t>(W) * CC) {
    const v4f* p[CC];
#pragma unroll
    for (int c = 0; c < CC; ++c)
      p[c] = reinterpret_cast<const v4f*>(psi32 + (c0 + c < ce ? c0 + c : c0) * ld);
    float acc[CC];
    dot_cols_f32<CC>(p, r_lds, ld4, lane, acc);
#pragma unroll
    for (int c = 0; c < CC; ++c) {
      if (c0 + c < ce) {
        const uint64_t k = make_key(acc[c], static_cast<int>(c0 + c));
        best = k > best ? k : best;
      }
    }
  }
  return best;
}

// BF16: each column's sum (dot_columns_lp's), inserted into L.
template <int CC>
__device__ inline void lp_pass_wave(const v4u* __restrict__ pq, int nq,
                                    const v4f* __restrict__ r_lds, int64_t cb, int64_t ce,
                                    int wave, int W, int lane, uint64_t (&L)[kTopK]) {
  for (int64_t c0 = cb + static_cast<int64_t>(wave) * CC; c0 < ce;
       c0 += static_cast<int64_t>(W) * CC) {
    const v4u* p[CC];
#pragma unroll
    for (int c = 0; c < CC; ++c) p[c] = pq + (c0 + c < ce ? c0 + c : c0) * nq;
    float acc[CC];
    dot_cols_lp<CC>(p, r_lds, nq, lane, acc);
#pragma unroll
    for (int c = 0; c < CC; ++c)
      if (c0 + c < ce) top8_insert(L, make_key(acc[c], static_cast<int>(c0 + c)));
  }
}

// ---- short columns: several side by side in one wave -----------------------
//
// A column of at most G 16-byte elements (G = 16 or 32) leaves most of a
// wave idle and its sum alone on the critical path.  These passes put
// P = 64/G columns side by side: lane group h (lanes h*G .. h*G+G-1) takes
// column c0 + c*P + h, each lane one element, as the wave-wide form has at
// these sizes.  group_sum takes the first steps of wave_sum, whose later
// steps there only add the other lanes' zeros, so every sum, and so every
// key, is the wave-wide form's bit for bit.  Each group keeps its own best
// key (FP32) or top-8 list (BF16); the lists are merged into one per wave at
// the end of the pass, the best keys by the workgroup's max, so the
// workgroup-wide result is the wave-wide form's.

template <int G>
__device__ inline float group_sum(float v) {
  static_assert(G == 16 || G == 32, "lane groups of 16 or 32");
  v += dpp_f32<kDppQuadSwap1>(v);
  v += dpp_f32<kDppQuadSwap2>(v);
  v += dpp_f32<kDppRowMirror>(v);
  v += dpp_f32<kDppRowHalfMirror>(v);
  if constexpr (G == 32) v += __shfl_xor(v, 16, kWave);
  return v;
}

// FP32 columns of ld4 <= G elements; returns the best key of this lane
// group's columns (lanes differ).
template <int G, int CC>
__device__ inline uint64_t f32_pass_grouped(const float* __restrict__ psi32, int64_t ld, int ld4,
                                            const v4f* __restrict__ r_lds, int64_t cb,
                                            int64_t ce, int wave, int W, int lane) {
  constexpr int P = kWave / G;
  const int h = lane / G, sl = lane % G;
  uint64_t best = 0;
  for (int64_t c0 = cb + static_cast<int64_t>(wave) * P * CC; c0 < ce;
       c0 += static_cast<int64_t>(W) * P * CC) {
    float acc[CC];
#pragma unroll
    for (int c = 0; c < CC; ++c) acc[c] = 0.0f;
    if (sl < ld4) {
      const v4f b = r_lds[sl];
#pragma unroll
      for (int c = 0; c < CC; ++c) {
        const int64_t col = c0 + c * P + h;
        const v4f a = __builtin_nontemporal_load(
            reinterpret_cast<const v4f*>(psi32 + (col < ce ? col : c0) * ld) + sl);
        acc[c] = __builtin_fmaf(a.x, b.x, acc[c]);
        acc[c] = __builtin_fmaf(a.y, b.y, acc[c]);
        acc[c] = __builtin_fmaf(a.z, b.z, acc[c]);
        acc[c] = __builtin_fmaf(a.w, b.w, acc[c]);
      }
    }
#pragma unroll
    for (int c = 0; c < CC; ++c) {
      const int64_t col = c0 + c * P + h;
      const uint64_t k = make_key(group_sum<G>(acc[c]), static_cast<int>(col));
      if (col < ce) best = k > best ? k : best;
    }
  }
  return best;
}

// BF16 columns of nq <= G elements, each with dot_columns_lp's arithmetic;
// leaves this wave's 8 best in L, the same in every lane.
template <int G, int CC>
__device__ inline void lp_pass_grouped(const v4u* __restrict__ pq, int nq,
                                       const v4f* __restrict__ r_lds, int64_t cb, int64_t ce,
                                       int wave, int W, int lane, uint64_t (&L)[kTopK]) {
  constexpr int P = kWave / G;
  const int h = lane / G, sl = lane % G;
  for (int64_t c0 = cb + static_cast<int64_t>(wave) * P * CC; c0 < ce;
       c0 += static_cast<int64_t>(W) * P * CC) {
    const v4u* p[CC];
#pragma unroll
    for (int c = 0; c < CC; ++c) {
      const int64_t col = c0 + c * P + h;
      p[c] = pq + (col < ce ? col : c0) * nq;
    }
    float acc[CC];
#pragma unroll
    for (int c = 0; c < CC; ++c) acc[c] = 0.0f;
    if (sl < nq) {
      int i = sl;
      lp_block_cols<2, 1, CC>(p, r_lds, i, acc);
    }
#pragma unroll
    for (int c = 0; c < CC; ++c) {
      const int64_t col = c0 + c * P + h;
      const uint64_t k = make_key(group_sum<G>(acc[c]), static_cast<int>(col));
      if (col < ce) top8_insert(L, k);
    }
  }
  // the groups' lists into one: group 0's, then the others' entries inserted
  uint64_t M[kTopK];
#pragma unroll
  for (int j = 0; j < kTopK; ++j) M[j] = lane_u64(L[j], 0);
#pragma unroll
  for (int g = 1; g < P; ++g)
#pragma unroll
    for (int j = 0; j < kTopK; ++j) top8_insert(M, lane_u64(L[j], g * G));
#pragma unroll
  for (int j = 0; j < kTopK; ++j) L[j] = M[j];
}

// Before a decode: the work list from its start, no failure, record slots
// zero (a plain fill, so that the decode can be captured in a graph).
__global__ __launch_bounds__(256) void k_ragged_reset(RQueue* q, unsigned long long* slots,
                                                      int64_t nwords) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    q->next = 0u;
    q->fail = 0;
  }
  const int64_t stride = static_cast<int64_t>(gridDim.x) * 256;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < nwords; i += stride)
    slots[i] = 0ull;
}

// Publish this part's record of step t (kTopK keys in lanes 0..kTopK-1 of
// wave 0, or one key in lane 0) and gather the parts' records into lanes
// (part * kTopK + j) of wave 0; keys past a part's count are 0.  Called by
// wave 0 only.  Returns false when a wait gave up (the queue's fail word is
// then set).
template <int K>
__device__ inline bool ragged_exchange(uint64_t mine, int lane, int part, int parts,
                                       unsigned long long* __restrict__ rec, long long t,
                                       long long spin_limit, RQueue* __restrict__ q,
                                       uint64_t& got) {
  const unsigned long long tag = static_cast<unsigned long long>(static_cast<unsigned>(t + 1))
                                 << 32;
  unsigned long long* half = rec + (t & 1) * kRaggedMaxParts * kRaggedRecWords;
  if (lane < K) {
    unsigned long long* w = half + part * kRaggedRecWords + 2 * lane;
    __hip_atomic_store(w, tag | (mine >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(w + 1, tag | (mine & 0xFFFFFFFFull), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
  got = 0;
  bool ok = true;
  const int pq = lane / K, j = lane % K;
  if (pq < parts && (K > 1 || lane < parts)) {
    unsigned long long* w = half + pq * kRaggedRecWords + 2 * j;
    long long spins = 0;
    for (;;) {
      if (spins >= spin_limit) {
        ok = false;
        break;
      }
      const unsigned long long lo = __hip_atomic_load(w + 1, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
      if ((lo >> 32) == (tag >> 32)) {
        const unsigned long long hi = __hip_atomic_load(w, __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT);
        if ((hi >> 32) == (tag >> 32)) {
          got = ((hi & 0xFFFFFFFFull) << 32) | (lo & 0xFFFFFFFFull);
          break;
        }
      }
      ++spins;
      __builtin_amdgcn_s_sleep(1);
    }
  }
  ok = __all(ok);
  if (!ok && lane == 0)
    (void)__hip_atomic_fetch_or(&q->fail, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return ok;
}

template <int NT, int CC, bool LP>
__global__ __launch_bounds__(NT) void k_ragged(const RInst* __restrict__ inst,
                                               const RItem* __restrict__ items, int nitems,
                                               const float* __restrict__ Y,
                                               float* __restrict__ X, float* __restrict__ R,
                                               const long long* __restrict__ caps,
                                               long long cap_all, double eps, int rescore_k,
                                               RResult* __restrict__ res,
                                               RQueue* __restrict__ q,
                                               unsigned long long* __restrict__ slots,
                                               long long spin_limit, mp_trace tr) {
  constexpr int W = NT / kWave;
  extern __shared__ v4f r_lds[];
  float* rf = reinterpret_cast<float*>(r_lds);
  __shared__ uint64_t kred[W];
  __shared__ double dred[W];
  __shared__ uint64_t lists[16 * kTopK];  // LP: per-wave top-8 lists (zero padded)
  __shared__ uint64_t cand[kTopK];
  __shared__ uint64_t resc[kTopK];
  __shared__ uint64_t s_best;
  __shared__ int s_item, s_ok;
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;

  for (;;) {
    if (threadIdx.x == 0)
      s_item = static_cast<int>(
          __hip_atomic_fetch_add(&q->next, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    __syncthreads();
    const int item = s_item;
    __syncthreads();  // s_item is rewritten next time round
    if (item >= nitems) break;
    const RItem it = items[item];
    const int id = it.id, part = it.part, parts = it.parts;
    const RInst d = inst[id];
    const int64_t n = d.n, m = d.m, ld = d.ld;
    const int ld4 = static_cast<int>(ld / 4);
    const float* y = Y + d.y_off;
    float* x = X + d.x_off;
    // this part's columns
    const int64_t cb = m * part / parts, ce = m * (part + 1) / parts;
    unsigned long long* rec =
        parts > 1 ? slots + static_cast<int64_t>(it.slot) * 2 * kRaggedMaxParts * kRaggedRecWords
                  : nullptr;
    const bool lead = part == 0;  // writes x~, the trace, r and the result

    // ---- init (eq. 8) ----
    if (lead)
      for (int64_t j = threadIdx.x; j < m; j += NT) x[j] = 0.0f;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < ld; i += NT) {
      const float v = i < n ? y[i] : 0.0f;
      rf[i] = v;
      s += static_cast<double>(v) * v;
    }
    const double yy = block_sum<NT>(s, dred);
    const double thr = eps * eps * yy;
    const long long T = caps ? caps[id] : cap_all;
    double rr = yy;
    long long t = 0;
    int reason;
    if (!__builtin_isfinite(yy)) {
      reason = kStopNonFinite;
    } else if (yy == 0.0) {
      reason = MP_STOP_ZERO_INPUT;
    } else {
      for (;;) {
        if (!(rr > thr)) {
          reason = MP_STOP_CONVERGED;
          break;
        }
        if (t >= T) {
          reason = MP_STOP_MAX_ITERS;
          break;
        }
        // ---- correlation pass (eq. 9) over this part's columns and argmax ----
        uint64_t best = 0;
        if constexpr (!LP) {
          if (ld4 <= 16)
            best = f32_pass_grouped<16, CC>(d.psi32, ld, ld4, r_lds, cb, ce, wave, W, lane);
          else if (ld4 <= 32)
            best = f32_pass_grouped<32, CC>(d.psi32, ld, ld4, r_lds, cb, ce, wave, W, lane);
          else
            best = f32_pass_wave<CC>(d.psi32, ld, ld4, r_lds, cb, ce, wave, W, lane);
          best = block_max<NT>(best, kred);
          if (parts > 1) {
            // the siblings' best keys of this step; the largest is the winner
            if (wave == 0) {
              uint64_t got = 0;
              const bool ok = ragged_exchange<1>(best, lane, part, parts, rec, t, spin_limit, q,
                                                 got);
              const uint64_t win = wave_max(got);
              if (lane == 0) {
                s_best = win;
                s_ok = ok ? 1 : 0;
              }
            }
            __syncthreads();
            best = s_best;
            if (!s_ok) {
              reason = kStopInternal;
              break;
            }
          }
        } else {
          const int nq = static_cast<int>(ld * 2 / 16);
          const v4u* pq = reinterpret_cast<const v4u*>(d.psib);
          uint64_t L[kTopK];
#pragma unroll
          for (int j = 0; j < kTopK; ++j) L[j] = 0;
          // (not at 1024 threads: with the grouped passes in, the 128
          // registers a lane has there spill in the wave-wide pass)
          bool grouped = false;
          if constexpr (NT <= 512) {
            grouped = nq <= 32;
            if (nq <= 16)
              lp_pass_grouped<16, CC>(pq, nq, r_lds, cb, ce, wave, W, lane, L);
            else if (nq <= 32)
              lp_pass_grouped<32, CC>(pq, nq, r_lds, cb, ce, wave, W, lane, L);
          }
          if (!grouped) lp_pass_wave<CC>(pq, nq, r_lds, cb, ce, wave, W, lane, L);
          uint64_t v = 0;
#pragma unroll
          for (int j = 0; j < kTopK; ++j)
            if (lane == j) v = L[j];
          if (lane < kTopK) lists[wave * kTopK + lane] = v;
          if (wave == 0)  // zero the unused list slots (W < 16)
            for (int k = W * kTopK + lane; k < 16 * kTopK; k += kWave) lists[k] = 0;
          __syncthreads();
          if (wave == 0) {
            uint64_t c8 = top8_of_lists16(lists[lane], lists[lane + kWave], lane);
            int ok = 1;
            if (parts > 1) {
              // the siblings' 8 best of this step, lanes 8 p + j, merged into
              // the instance's 8 best
              uint64_t got = 0;
              ok = ragged_exchange<kTopK>(c8, lane, part, parts, rec, t, spin_limit, q, got)
                       ? 1 : 0;
              c8 = top8_of_lists16(got, 0ull, lane);
            }
            if (lane < kTopK) cand[lane] = c8;
            if (lane == 0) s_ok = ok;
          }
          __syncthreads();
          if (parts > 1 && !s_ok) {
            reason = kStopInternal;
            break;
          }
          for (int qd = wave; qd < rescore_k; qd += W) {
            const uint64_t k = cand[qd];
            uint64_t rk = 0;
            if (k != 0) {
              const int idx = key_index(k);
              if (idx >= 0 && idx < m) {
                const float c32 = dot_column_f32<false>(
                    reinterpret_cast<const v4f*>(d.psi32 + static_cast<int64_t>(idx) * ld),
                    r_lds, ld4, lane);
                rk = make_key(c32, idx);
              }
            }
            if (lane == 0) resc[qd] = rk;
          }
          __syncthreads();
          for (int qd = 0; qd < rescore_k; ++qd) best = resc[qd] > best ? resc[qd] : best;
        }
        const int idx = key_index(best);
        const float c = key_value(best);
        if (best == 0 || idx < 0 || idx >= m) {
          reason = kStopInternal;
          break;
        }
        if (c == 0.0f) {
          reason = MP_STOP_STALLED;
          break;
        }
        // ---- update (eqs. 10-12); every wave is past the pass (barrier above) ----
        const float* colp = d.psi32 + static_cast<int64_t>(idx) * ld;
        float* rt = lead && tr.r && t < tr.cap
                        ? tr.r + (static_cast<int64_t>(id) * tr.cap + t) * tr.ldr : nullptr;
        s = 0.0;
        for (int64_t i = threadIdx.x; i < n; i += NT) {
          const float vv = __builtin_fmaf(-c, colp[i], rf[i]);
          rf[i] = vv;
          if (rt) rt[i] = vv;
          s += static_cast<double>(vv) * vv;
        }
        rr = block_sum<NT>(s, dred);  // its barriers publish the new r to all waves
        if (lead && threadIdx.x == 0) {
          x[idx] += c;
          if (t < tr.cap) {
            const int64_t o = static_cast<int64_t>(id) * tr.cap + t;
            if (tr.idx) tr.idx[o] = idx;
            if (tr.coef) tr.coef[o] = c;
            if (tr.rr) tr.rr[o] = rr;
          }
        }
        ++t;
      }
    }
    if (R && lead)
      for (int64_t i = threadIdx.x; i < n; i += NT) R[d.y_off + i] = rf[i];
    if (lead && threadIdx.x == 0) {
      RResult o;
      o.t = t;
      o.yy = yy;
      o.rr = rr;
      o.reason = reason;
      o.pad = 0;
      res[id] = o;
    }
    __syncthreads();  // r_lds and the LDS lists are reused by the next instance
  }
}

// ---------------------------------------------------------------------------

template <int NT, int CC, bool LP>
static hipError_t launch_ragged_t(int grid, size_t lds, const RInst* inst, const RItem* items,
                                  int nitems, const float* Y, float* X, float* R,
                                  const long long* caps, long long cap_all, double eps,
                                  int rescore_k, RResult* res, RQueue* q,
                                  unsigned long long* slots, long long spin_limit, mp_trace tr,
                                  hipStream_t s) {
  // instances have n <= 8192, so the residual needs at most 32 KB of LDS
  k_ragged<NT, CC, LP><<<dim3(grid), dim3(NT), lds, s>>>(inst, items, nitems, Y, X, R, caps,
                                                         cap_all, eps, rescore_k, res, q, slots,
                                                         spin_limit, tr);
  return hipGetLastError();
}

bool ragged_config_valid(const RConfig& cf, bool lp) {
  const bool nt_ok = cf.threads == 256 || cf.threads == 512 || cf.threads == 1024;
  const bool cc_ok = cf.cols_per_wave == 1 || cf.cols_per_wave == 2 || cf.cols_per_wave == 4;
  (void)lp;
  return nt_ok && cc_ok && cf.wgs_per_cu >= 1 && cf.wgs_per_cu <= 8 && cf.split >= 1 &&
         cf.split <= kRaggedMaxParts;
}

hipError_t launch_ragged(const RConfig& cf, bool lp, int grid, size_t lds, const RInst* inst,
                         const RItem* items, int nitems, const float* Y, float* X, float* R,
                         const long long* caps, long long cap_all, double eps, int rescore_k,
                         RResult* res, RQueue* q, unsigned long long* slots, int nslots,
                         long long spin_limit, mp_trace tr, hipStream_t s) {
  const int64_t nwords = static_cast<int64_t>(nslots) * 2 * kRaggedMaxParts * kRaggedRecWords;
  int64_t rb = (nwords + 255) / 256;
  rb = rb < 1 ? 1 : (rb > 256 ? 256 : rb);
  k_ragged_reset<<<dim3(static_cast<unsigned>(rb)), dim3(256), 0, s>>>(q, slots, nwords);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
#define MP_RAGGED_CASE(NT, CC, LP)                                                          \
  if (cf.threads == NT && cf.cols_per_wave == CC && lp == LP)                               \
    return launch_ragged_t<NT, CC, LP>(grid, lds, inst, items, nitems, Y, X, R, caps,        \
                                       cap_all, eps, rescore_k, res, q, slots, spin_limit, tr, \
                                       s);
  MP_RAGGED_CASE(256, 1, false)
  MP_RAGGED_CASE(256, 2, false)
  MP_RAGGED_CASE(256, 4, false)
  MP_RAGGED_CASE(512, 1, false)
  MP_RAGGED_CASE(512, 2, false)
  MP_RAGGED_CASE(512, 4, false)
  MP_RAGGED_CASE(1024, 1, false)
  MP_RAGGED_CASE(1024, 2, false)
  MP_RAGGED_CASE(1024, 4, false)
  MP_RAGGED_CASE(256, 1, true)
  MP_RAGGED_CASE(256, 2, true)
  MP_RAGGED_CASE(256, 4, true)
  MP_RAGGED_CASE(512, 1, true)
  MP_RAGGED_CASE(512, 2, true)
  MP_RAGGED_CASE(512, 4, true)
  MP_RAGGED_CASE(1024, 1, true)
  MP_RAGGED_CASE(1024, 2, true)
  MP_RAGGED_CASE(1024, 4, true)
#undef MP_RAGGED_CASE
  return hipErrorInvalidValue;
}

}  // namespace mp
