// Reduced-precision dictionary forms of the MP iteration for gfx950.
//
// The correlation pass (eq. 9) streams a BF16 copy of the dictionary, or an
// FP8 (OCP E4M3, "e4m3fn") copy with one FP32 scale per column, and
// accumulates in FP32 against the FP32 residual.  Because the reduced
// precision can reorder near-equal correlations, each pass keeps the 8 best
// candidates rather than 1; at the start of the next launch every workgroup
// re-scores up to 8 of them against the FP32 columns (the same FP32 inner
// product the FP32 form computes, each column's two chains on two waves) and
// takes the best of those, smallest index on ties (eq. 16).
// The coefficient and residual updates (eqs. 10-11) and the FP64 stopping
// test then use the FP32 column and the re-scored FP32 coefficient.
//
// Set-up quantisers:
//   BF16  round to nearest even of the FP32 value.
//   FP8   s_m = fp32(max_n |psi_nm| / 448) (1 for an all-zero column);
//         code = round-to-nearest-even of fp32(psi_nm / s_m), saturating at
//         +-448 (the largest finite e4m3fn value).
#include "k_common.h"
#include "k_lowp.h"
#include "mp_internal.h"

namespace mp {

constexpr int kLpThreads = 1024;
constexpr int kLpWaves = kLpThreads / kWave;
// Columns one wave streams at once: an FP8 column (N bytes) is short enough
// that two in flight together keep more of HBM busy.
template <int S>
constexpr int kLpColsPerWave = S == 1 ? 2 : 1;

// ---------------------------------------------------------------------------
// Quantisers

// FP32 -> e4m3fn code, round to nearest even, saturating at 448.
__device__ inline uint8_t fp8_e4m3_rne_sat(float v) {
  const uint32_t u = __builtin_bit_cast(uint32_t, v);
  const uint32_t sign = (u >> 24) & 0x80u;
  const float a = __builtin_fabsf(v);
  uint32_t code;
  if (!(a < 448.0f)) {
    code = 0x7Eu;  // saturate (a value at or above the largest finite one)
  } else if (a < 0.015625f) {
    // below 2^-6 the representable values are the multiples of 2^-9 (the
    // subnormals, then 2^-6 itself as code 8); a * 512 is exact
    code = static_cast<uint32_t>(__builtin_rintf(a * 512.0f));
  } else {
    const uint32_t au = __builtin_bit_cast(uint32_t, a);
    int e = static_cast<int>(au >> 23) - 127;  // -6 .. 8
    const uint32_t mant = au & 0x7FFFFFu;
    uint32_t m3 = mant >> 20;                   // 3 kept mantissa bits
    const uint32_t rem = mant & 0xFFFFFu;       // 20 dropped bits
    if (rem > 0x80000u || (rem == 0x80000u && (m3 & 1u))) ++m3;
    if (m3 == 8u) {
      m3 = 0u;
      ++e;
    }
    code = (static_cast<uint32_t>(e + 7) << 3) | m3;  // a < 448 keeps this <= 0x7E
  }
  return static_cast<uint8_t>(code | sign);
}

__global__ __launch_bounds__(256) void k_quant_bf16(const float* __restrict__ psi, int64_t count,
                                                    uint16_t* __restrict__ out) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
       i += stride)
    out[i] = bf16_rne(psi[i]);
}

// One wave per column: the column's largest |psi|, its scale, then the codes
// (padding rows hold 0 and get code 0).
__global__ __launch_bounds__(256) void k_quant_fp8(const float* __restrict__ psi, int64_t ld,
                                                   int64_t m, uint8_t* __restrict__ out,
                                                   float* __restrict__ scales) {
  const int lane = threadIdx.x % kWave;
  const int64_t col = static_cast<int64_t>(blockIdx.x) * 4 + threadIdx.x / kWave;
  if (col >= m) return;
  const float* p = psi + col * ld;
  float amax = 0.0f;
  for (int64_t i = lane; i < ld; i += kWave) amax = __builtin_fmaxf(amax, __builtin_fabsf(p[i]));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) amax = __builtin_fmaxf(amax, __shfl_xor(amax, off, kWave));
  const float s = amax == 0.0f ? 1.0f : amax / 448.0f;
  if (lane == 0) scales[col] = s;
  uint8_t* q = out + col * ld;
  for (int64_t i = lane; i < ld; i += kWave) q[i] = fp8_e4m3_rne_sat(p[i] / s);
}

hipError_t launch_quant_bf16(const float* psi, int64_t ld, int64_t m, uint16_t* out,
                             hipStream_t s) {
  const int64_t count = ld * m;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  k_quant_bf16<<<dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s>>>(psi, count, out);
  return hipGetLastError();
}

hipError_t launch_quant_fp8(const float* psi, int64_t ld, int64_t m, uint8_t* out,
                            float* scales, hipStream_t s) {
  const int64_t blocks = (m + 3) / 4;
  k_quant_fp8<<<dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s>>>(psi, ld, m, out, scales);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// One MP iteration with a reduced-precision correlation pass (one launch),
// the selection carried into the next launch so that no workgroup waits for
// another (no hand-off through atomics, no single-workgroup tail).
//
// Launch k (k >= 1) finishes step k and runs pass k+1:
//  1. every workgroup requests at once r_{k-1} (half k mod 2 of rbuf) and
//     the 8 keys each workgroup of launch k-1 stored;
//  2. every workgroup merges the published keys into the top 8, re-scores up
//     to `rescore_k` of them against the FP32 columns (two waves per
//     candidate, the FP32 form's inner product bit for bit), takes the best
//     re-scored candidate (idx, c) and updates its LDS copy of r,
//     r_k = r_{k-1} - c psi_idx with the FP32 column (eq. 11), and ||r_k||^2
//     in FP64 -- the same values in every workgroup, so the same stop test;
//  3. workgroup 0 alone stores r_k (the other half of rbuf), adds c to x~_idx
//     (eq. 10), writes the trace entry and the state (t = k, eq. 12);
//  4. unless the run stops here, every workgroup runs the reduced-precision
//     pass over its columns against r_k, keeps a top-8 list per wave, merges
//     its 16 lists and stores 8 keys for launch k+1.
// Launch 0 runs the first pass on r = y (workgroup 0 copies r to the other
// half); T steps take T+1 launches.  Same shape as the FP32 step: 16-wave
// workgroups, wave w of workgroup b takes columns b*cpw + w, + 16, ...
// (FP8: pairs b*cpw + 2w, 2w + 1, + 32, ...).
template <int S>
__global__ __launch_bounds__(kLpThreads) void k_mp_step_lp(
    const v4u* __restrict__ psiq, const float* __restrict__ scales,
    const float* __restrict__ psi32, int64_t ld, int64_t n, int64_t m, float* __restrict__ rbuf,
    int cols_per_wg, int rescore_k, uint64_t* __restrict__ keys, long long k,
    long long max_iters, float* __restrict__ x, DevState* __restrict__ st,
    mp_trace tr) {
  extern __shared__ v4f r_lds[];
  __shared__ uint64_t lists[kLpWaves * kTopK];
  __shared__ uint64_t cand[kTopK];
  __shared__ uint64_t rescored[kTopK];
  __shared__ float chain_b[kTopK][kWave];
  __shared__ double dred[kLpWaves];
  __shared__ int s_done;
  constexpr int CC = kLpColsPerWave<S>;
  constexpr int RPT = 16384 / 4 / kLpThreads;  // float4s of r per thread (ld <= 16384)
  const int ld4 = static_cast<int>(ld / 4);
  const int nq = static_cast<int>(ld * S / 16);
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int par = static_cast<int>(k & 1);
  const bool first = k == 0;
  const v4f* r_in = reinterpret_cast<const v4f*>(rbuf + (par ? ld : 0));
  v4f* r_out = reinterpret_cast<v4f*>(rbuf + (par ? 0 : ld));
  const int nslots = static_cast<int>(gridDim.x) * kTopK;  // <= 2 * kLpThreads (host-checked)
  const uint64_t* k_in = keys + (par ? nslots : 0);
  uint64_t* k_out = keys + (par ? 0 : nslots);
  const int64_t col0 = static_cast<int64_t>(blockIdx.x) * cols_per_wg;
  int64_t col1 = col0 + cols_per_wg;
  if (col1 > m) col1 = m;

  // ---- 1. requests (clamped indices into valid memory, unused values dropped)
  int done_v = 0;
  if (threadIdx.x == 0)
    done_v = __hip_atomic_load(&st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // eps^2 ||y||^2, set by the init kernel before the first launch
  const double thr = st->thr;
  v4f rq[RPT];
#pragma unroll
  for (int u = 0; u < RPT; ++u) {
    const int i = threadIdx.x + u * kLpThreads;
    rq[u] = r_in[i < ld4 ? i : ld4 - 1];
  }
  const int ia = threadIdx.x < nslots ? threadIdx.x : nslots - 1;
  const int ib = threadIdx.x + kLpThreads < nslots ? threadIdx.x + kLpThreads : nslots - 1;
  uint64_t ka = k_in[ia], kb = k_in[ib];
  if (first || threadIdx.x >= static_cast<unsigned>(nslots)) ka = 0;
  if (first || threadIdx.x + kLpThreads >= static_cast<unsigned>(nslots)) kb = 0;
#pragma unroll
  for (int u = 0; u < RPT; ++u) {
    const int i = threadIdx.x + u * kLpThreads;
    if (i < ld4) r_lds[i] = rq[u];
  }
  if (threadIdx.x == 0) s_done = done_v;
  __syncthreads();
  if (s_done) return;

  if (!first) {
    // ---- 2. the top 8 of the published keys (slot 8g + j holds workgroup g's
    // rank-j key, so every group of 8 lanes holds one sorted list) ----
    const uint64_t wtop = top8_of_lists16(ka, kb, lane);
    if (lane < kTopK) lists[wave * kTopK + lane] = wtop;
    __syncthreads();
    if (wave == 0) {
      const uint64_t t = top8_of_lists16(lists[lane], lists[lane + kWave], lane);
      if (lane < kTopK) cand[lane] = t;
    }
    __syncthreads();
    // re-score: waves 2q and 2q+1 run the two chains of candidate q's inner
    // product, which meet per lane in LDS
    static_assert(kLpWaves >= 2 * kTopK, "two waves per candidate");
    {
      const int q = wave / 2;
      const bool second = (wave % 2) != 0;
      const int h0 = ld4 / 2;
      int idx = -1;
      if (q < rescore_k && cand[q] != 0) {
        idx = key_index(cand[q]);
        if (idx >= m) idx = -1;
      }
      float acc = 0.0f;
      if (idx >= 0) {
        acc = dot_chain_f32(reinterpret_cast<const v4f*>(psi32 + static_cast<int64_t>(idx) * ld),
                            r_lds, second ? h0 : 0, h0, lane);
        if (second) chain_b[q][lane] = acc;
      }
      __syncthreads();
      if (!second && q < rescore_k) {
        uint64_t rk = 0;
        if (idx >= 0) rk = make_key(wave_sum(acc + chain_b[q][lane]), idx);
        if (lane == 0) rescored[q] = rk;
      }
    }
    __syncthreads();
    uint64_t best = 0;
    for (int j = 0; j < rescore_k; ++j) best = rescored[j] > best ? rescored[j] : best;
    const int idx = key_index(best);
    const float c = key_value(best);
    if (carried_winner_stops(idx, c, m, st)) return;
    if (carried_update<kLpThreads>(idx, c, psi32, ld, n, r_lds, r_out, x, st, tr, k, max_iters, thr,
                                   par ^ 1, dred))
      return;
  } else if (blockIdx.x == 0) {
    for (int i = threadIdx.x; i < ld4; i += kLpThreads) r_out[i] = r_lds[i];
    if (threadIdx.x == 0) st->r_sel = par ^ 1;
  }

  // ---- 4. the pass against r_k ----
  uint64_t L[kTopK];
#pragma unroll
  for (int j = 0; j < kTopK; ++j) L[j] = 0;
  // wave w takes columns in runs of CC: col0 + CC*w, ..., then + CC*16
  for (int64_t col = col0 + CC * wave; col < col1; col += CC * kLpWaves) {
    const v4u* p[CC];
#pragma unroll
    for (int c = 0; c < CC; ++c) p[c] = psiq + (col + c < col1 ? col + c : col) * nq;
    float cv[CC];
    dot_columns_lp<S, CC>(p, r_lds, nq, lane, cv);
#pragma unroll
    for (int c = 0; c < CC; ++c) {
      if (col + c < col1) {
        float v = cv[c];
        if constexpr (S == 1) v *= scales[col + c];
        top8_insert(L, make_key(v, static_cast<int>(col + c)));
      }
    }
  }
  {
    uint64_t v = 0;
#pragma unroll
    for (int j = 0; j < kTopK; ++j)
      if (lane == j) v = L[j];
    if (lane < kTopK) lists[wave * kTopK + lane] = v;
  }
  __syncthreads();
  if (wave == 0) {
    const uint64_t mine = top8_of_lists16(lists[lane], lists[lane + kWave], lane);
    if (lane < kTopK) k_out[blockIdx.x * kTopK + lane] = mine;
  }
}

hipError_t launch_mp_step_lp(mp_dtype storage, const void* psiq, const float* scales,
                             const float* psi32, int64_t ld, int64_t n, int64_t m, float* rbuf,
                             const CorrGeom& g, int rescore_k, uint64_t* keys, long long k,
                             long long max_iters, float* x, DevState* st,
                             mp_trace tr, hipStream_t s) {
  const size_t lds = static_cast<size_t>(ld) * sizeof(float);
  const v4u* q = static_cast<const v4u*>(psiq);
  static bool big_lds[2] = {false, false};
  const void* fn = storage == MP_BF16 ? reinterpret_cast<const void*>(k_mp_step_lp<2>)
                                      : reinterpret_cast<const void*>(k_mp_step_lp<1>);
  const int which = storage == MP_BF16 ? 0 : 1;
  if (!big_lds[which] && lds > 60 * 1024) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
    if (e != hipSuccess) return e;
    big_lds[which] = true;
  }
  if (storage == MP_BF16)
    k_mp_step_lp<2><<<dim3(g.grid), dim3(kLpThreads), lds, s>>>(
        q, nullptr, psi32, ld, n, m, rbuf, g.cols_per_wg, rescore_k, keys, k, max_iters, x,
        st, tr);
  else
    k_mp_step_lp<1><<<dim3(g.grid), dim3(kLpThreads), lds, s>>>(
        q, scales, psi32, ld, n, m, rbuf, g.cols_per_wg, rescore_k, keys, k, max_iters, x,
        st, tr);
  return hipGetLastError();
}

}  // namespace mp
