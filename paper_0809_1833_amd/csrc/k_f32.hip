// FP32 single-signal Matching Pursuit kernels for gfx950 (Section 3, eqs. 8-12).
//
// One MP iteration is one launch of k_mp_step_f32 on the caller's stream:
// c_m = <r, psi_m> for every column (eq. 9), streaming the whole column-major
// dictionary once with a per-workgroup argmax (largest |c_m|, smallest index
// on ties, eq. 16); the last workgroup to finish then picks i, updates
// x~_i += c_i (eq. 10) and r -= c_i psi_i (eq. 11), counts t (eq. 12) and runs
// the FP64 stopping test.  A launch returns at once when the device state says
// the run has stopped, so the host can enqueue iterations ahead without
// reading anything back.
#include "k_common.h"
#include "mp_internal.h"

namespace mp {

typedef float v4f __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Column norms (set-up check of eq. 4): norm2[m] = sum_n psi_nm^2 in FP64.
// One wave per column.
__global__ __launch_bounds__(256) void k_norms(const float* __restrict__ psi, int64_t ld,
                                               int64_t n, int64_t m,
                                               double* __restrict__ norm2) {
  const int lane = threadIdx.x % kWave;
  const int64_t col = static_cast<int64_t>(blockIdx.x) * 4 + threadIdx.x / kWave;
  if (col >= m) return;
  const float* p = psi + col * ld;
  double s = 0.0;
  for (int64_t i = lane; i < n; i += kWave) {
    double v = p[i];
    s += v * v;
  }
  s = wave_sum(s);
  if (lane == 0) norm2[col] = s;
}

hipError_t launch_norms(const float* psi, int64_t ld, int64_t n, int64_t m, double* norm2,
                        int* /*unused*/, hipStream_t s) {
  const int64_t blocks = (m + 3) / 4;
  k_norms<<<dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s>>>(psi, ld, n, m, norm2);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Init (eq. 8): r = y (zero padded to ld), x~ = 0, t = 0, ||y||^2 in FP64, and
// the pre-test of the loop for t = 0.
__global__ __launch_bounds__(256) void k_init(const float* __restrict__ y, int64_t n, int64_t ld,
                                              float* __restrict__ x, int64_t m,
                                              float* __restrict__ r, DevState* __restrict__ st,
                                              double eps, long long max_iters) {
  __shared__ double red[4];
  const int64_t gtid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t gstride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t j = gtid; j < m; j += gstride) x[j] = 0.0f;
  if (blockIdx.x != 0) return;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < ld; i += 256) {
    float v = i < n ? y[i] : 0.0f;
    r[i] = v;
    s += static_cast<double>(v) * v;
  }
  const double yy = block_sum<256>(s, red);
  if (threadIdx.x == 0) {
    DevState d{};
    d.yy = yy;
    d.rr = yy;
    d.thr = eps * eps * yy;
    d.t = 0;
    d.max_iters = max_iters;
    d.done = 0;
    d.reason = MP_STOP_CONVERGED;
    if (!__builtin_isfinite(yy)) {
      d.done = 1;
      d.reason = kStopNonFinite;
    } else if (yy == 0.0) {
      d.done = 1;
      d.reason = MP_STOP_ZERO_INPUT;
    } else if (!(yy > d.thr)) {
      d.done = 1;
      d.reason = MP_STOP_CONVERGED;
    } else if (max_iters <= 0) {
      d.done = 1;
      d.reason = MP_STOP_MAX_ITERS;
    }
    *st = d;
  }
}

hipError_t launch_init(const float* y, int64_t n, int64_t ld, float* x, int64_t m, float* r,
                       DevState* st, double eps, long long max_iters, hipStream_t s) {
  int64_t blocks = (m + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  k_init<<<dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s>>>(y, n, ld, x, m, r, st, eps,
                                                                    max_iters);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// One MP iteration in one launch (eqs. 9-12).
//
// Workgroup = 16 waves, one per CU.  The residual (ld floats, zero padded) is
// staged once into LDS; wave w of workgroup b takes columns b*cpw + w, + 16, ... and
// streams each column with 16-byte non-temporal loads (lane l reads float4s
// l, l+64, ...), UNROLL loads in flight per lane, FP32 FMA accumulation,
// then a butterfly sum across the wave.  Keys are max-reduced per wave and
// across the 16 waves; each workgroup publishes its key and counts itself in.  The workgroup that arrives last (nobody waits: it is
// simply the one that sees the count reach the grid size) takes the winning
// key, updates x~ and r, computes ||r||^2 in FP64 and applies the stopping
// test.
constexpr int kCorrThreads = 1024;
constexpr int kCorrUnroll = 16;

// U loads of 16 bytes in flight per lane, then U x 4 FMAs against the LDS
// copy of r; advances i by 64 * U float4s.
template <int U>
__device__ inline void dot_block(const v4f* __restrict__ p, const v4f* __restrict__ r_lds,
                                 int& i, float& acc) {
  v4f a[U];
#pragma unroll
  for (int u = 0; u < U; ++u) a[u] = __builtin_nontemporal_load(p + i + kWave * u);
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

// <r, psi_col> for one column by one wave: blocks of 16 loads per lane while
// they fit, then at most one block each of 8, 4, 2 and 1 (so short columns
// still have several loads in flight), then a butterfly sum.
__device__ inline float dot_column_f32(const v4f* __restrict__ p, const v4f* __restrict__ r_lds,
                                       int ld4, int lane) {
  float acc = 0.0f;
  int i = lane;
  while (i + kWave * (kCorrUnroll - 1) < ld4) dot_block<kCorrUnroll>(p, r_lds, i, acc);
  if (i + kWave * 7 < ld4) dot_block<8>(p, r_lds, i, acc);
  if (i + kWave * 3 < ld4) dot_block<4>(p, r_lds, i, acc);
  if (i + kWave * 1 < ld4) dot_block<2>(p, r_lds, i, acc);
  if (i < ld4) dot_block<1>(p, r_lds, i, acc);
  return wave_sum(acc);
}

// Selection and update, run by the last workgroup of a launch (NT threads).
// `best` is the launch's winning key (largest |c|, smallest index).
template <int NT>
__device__ void select_update_tail(uint64_t best, const float* __restrict__ psi, int64_t ld,
                                   int64_t n, int64_t m, float* __restrict__ x,
                                   float* __restrict__ r, DevState* __restrict__ st,
                                   const mp_trace& tr, double* dred) {
  const int idx = key_index(best);
  const float c = key_value(best);
  if (idx < 0 || idx >= m) {  // cannot happen for a key a workgroup published
    if (threadIdx.x == 0) {
      st->done = 1;
      st->reason = kStopInternal;
    }
    return;
  }
  if (c == 0.0f) {  // no atom correlates with r: MP cannot make progress
    if (threadIdx.x == 0) {
      st->done = 1;
      st->reason = MP_STOP_STALLED;
    }
    return;
  }
  const float* col = psi + static_cast<int64_t>(idx) * ld;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += NT) {
    const float v = __builtin_fmaf(-c, col[i], r[i]);
    r[i] = v;
    s += static_cast<double>(v) * v;
  }
  const double rr = block_sum<NT>(s, dred);
  if (threadIdx.x == 0) {
    x[idx] += c;
    const long long t = st->t;
    if (t < tr.cap) {
      if (tr.idx) tr.idx[t] = idx;
      if (tr.coef) tr.coef[t] = c;
      if (tr.rr) tr.rr[t] = rr;
    }
    st->t = t + 1;
    st->rr = rr;
    if (!(rr > st->thr)) {
      st->done = 1;
      st->reason = MP_STOP_CONVERGED;
    } else if (t + 1 >= st->max_iters) {
      st->done = 1;
      st->reason = MP_STOP_MAX_ITERS;
    }
  }
}

// Publish a workgroup's key and count the workgroup in; returns true in the
// workgroup that arrives last, together with the launch's winning key.
//
// The key slots and the arrival counter are only ever touched with atomic
// read-modify-write operations at device scope.  Each one is performed at
// the device's point of coherence for atomics and returns only once
// performed, and every RMW returns the latest value of its word.  A
// workgroup swaps its key into its own slot, waits for that swap to return,
// then increments the counter; the workgroup whose increment returns grid-1
// issues its reads after that, so each of its swaps-with-zero returns the
// key stored in this launch (and leaves the slot cleared for the next one).
// Plain or relaxed loads are not used for these words: a relaxed load is not
// ordered after the other workgroups' RMWs and could return an older value.
// No cache write-back or invalidate is needed; everything else the tail
// reads was written by earlier launches.
template <int NT>
__device__ inline bool publish_and_arrive(uint64_t key, uint64_t* keys, DevState* st,
                                          uint64_t* kred, uint64_t* winner) {
  __shared__ int s_last;
  if (threadIdx.x == 0) {
    const uint64_t old =
        __hip_atomic_exchange(keys + blockIdx.x, key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // Keys never have bit 63 set, so inc is 1; computing it from `old` makes
    // the increment wait for the exchange to have been performed.
    const unsigned inc = 1u + static_cast<unsigned>(old >> 63);
    const unsigned prev =
        __hip_atomic_fetch_add(&st->arrive, inc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int last = prev == gridDim.x - 1;
    if (last)
      (void)__hip_atomic_exchange(&st->arrive, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_last = last;
  }
  __syncthreads();
  if (!s_last) return false;
  uint64_t best = 0;
  for (int i = threadIdx.x; i < static_cast<int>(gridDim.x); i += NT) {
    const uint64_t k =
        __hip_atomic_exchange(keys + i, uint64_t{0}, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    best = k > best ? k : best;
  }
  *winner = block_max<NT>(best, kred);
  return true;
}

__global__ __launch_bounds__(kCorrThreads) void k_mp_step_f32(
    const float* __restrict__ psi, int64_t ld, int64_t n, int64_t m, float* __restrict__ r,
    int cols_per_wg, uint64_t* __restrict__ keys, float* __restrict__ x,
    DevState* __restrict__ st, mp_trace tr) {
  if (st->done) return;
  extern __shared__ v4f r_lds[];
  __shared__ uint64_t kred[kCorrThreads / kWave];
  __shared__ double dred[kCorrThreads / kWave];
  const int ld4 = static_cast<int>(ld / 4);
  const v4f* r4 = reinterpret_cast<const v4f*>(r);
  for (int i = threadIdx.x; i < ld4; i += kCorrThreads) r_lds[i] = r4[i];
  __syncthreads();

  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int64_t col0 = static_cast<int64_t>(blockIdx.x) * cols_per_wg;
  int64_t col1 = col0 + cols_per_wg;
  if (col1 > m) col1 = m;
  uint64_t best = 0;
  for (int64_t col = col0 + wave; col < col1; col += kCorrThreads / kWave) {
    const float c = dot_column_f32(reinterpret_cast<const v4f*>(psi + col * ld), r_lds, ld4, lane);
    const uint64_t k = make_key(c, static_cast<int>(col));
    best = k > best ? k : best;
  }
  best = block_max<kCorrThreads>(best, kred);
  uint64_t winner = 0;
  if (!publish_and_arrive<kCorrThreads>(best, keys, st, kred, &winner)) return;
  select_update_tail<kCorrThreads>(winner, psi, ld, n, m, x, r, st, tr, dred);
}

CorrGeom corr_f32_geometry(int64_t m, int num_cus) {
  // One 16-wave workgroup per CU (one LDS copy of r per CU, few arrivals);
  // a workgroup takes at least one column per wave.
  constexpr int64_t kWaves = kCorrThreads / kWave;
  const int64_t target = num_cus > 0 ? num_cus : 256;
  int64_t cpw = (m + target - 1) / target;
  cpw = ((cpw + kWaves - 1) / kWaves) * kWaves;
  if (cpw < kWaves) cpw = kWaves;
  CorrGeom g;
  g.cols_per_wg = static_cast<int>(cpw);
  g.grid = static_cast<int>((m + cpw - 1) / cpw);
  return g;
}

hipError_t launch_mp_step_f32(const float* psi, int64_t ld, int64_t n, int64_t m, float* r,
                              const CorrGeom& g, uint64_t* keys, float* x, DevState* st,
                              mp_trace tr, hipStream_t s) {
  const size_t lds = static_cast<size_t>(ld) * sizeof(float);
  static bool big_lds = false;  // residuals above 60 KB need the opt-in limit
  if (!big_lds && lds > 60 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_mp_step_f32),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
    if (e != hipSuccess) return e;
    big_lds = true;
  }
  k_mp_step_f32<<<dim3(g.grid), dim3(kCorrThreads), lds, s>>>(psi, ld, n, m, r, g.cols_per_wg,
                                                              keys, x, st, tr);
  return hipGetLastError();
}

}  // namespace mp
