// FP32 single-signal Matching Pursuit kernels for gfx950 (Section 3, eqs. 8-12).
//
// One MP step per launch of k_mp_step_f32 on the caller's stream: launch k
// applies step k (the winner of launch k-1's pass: x~_i += c_i, eq. 10;
// r -= c_i psi_i, eq. 11; t = k, eq. 12; the FP64 stopping test) and then
// computes c_m = <r, psi_m> for every column (eq. 9), streaming the whole
// column-major dictionary once with a per-workgroup argmax (largest |c_m|,
// smallest index on ties, eq. 16).  A launch returns at once when the device
// state says the run has stopped, so the host can enqueue launches ahead
// without reading anything back.
#include <stdlib.h>

#include <algorithm>

#include "k_common.h"
#include "mp_internal.h"

namespace mp {

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
// One MP iteration per launch (eqs. 9-12), the selection carried into the
// next launch so that no workgroup waits for another.
//
// Workgroup = 16 waves, one per CU.  Launch k (k >= 1): every workgroup
// stages r_{k-1} (half k mod 2 of the residual buffer, ld floats, zero
// padded) into LDS and reads the keys the workgroups of launch k-1 stored
// (the kernel boundary orders them); all take the same winner (largest |c|,
// smallest index, eq. 16), apply step k to their LDS copy of r and compute
// ||r_k||^2 in FP64 (carried_update: workgroup 0 also stores r_k in the
// other half and keeps x~, the trace and the state); unless the run stops
// there, each runs pass k+1 over its share of the columns (balanced between
// the XCDs from the previous launch's timings): wave w takes columns
// col0 + w, + 16, ... and streams each column with 16-byte non-temporal
// loads (two per-lane FP32 FMA chains over the column halves, then a
// butterfly sum across the wave), keys are max-reduced per wave and across
// the 16 waves, and the workgroup stores its key for launch k+1.  Launch 0
// runs the first pass on r = y; T steps take T+1 launches.
constexpr int kCorrThreads = 1024;

__global__ __launch_bounds__(kCorrThreads) void k_mp_step_f32(
    const float* __restrict__ psi, int64_t ld, int64_t n, int64_t m, float* __restrict__ rbuf,
    int cols_per_wg, uint64_t* __restrict__ keys, BalState* __restrict__ bal, long long k,
    long long max_iters, float* __restrict__ x, DevState* __restrict__ st,
    mp_trace tr) {
  extern __shared__ v4f r_lds[];
  __shared__ uint64_t kred[kCorrThreads / kWave];
  __shared__ double dred[kCorrThreads / kWave];
  __shared__ int s_done;
  constexpr int RPT = 16384 / 4 / kCorrThreads;  // float4s of r per thread (ld <= 16384)
  const int ld4 = static_cast<int>(ld / 4);
  const int par = static_cast<int>(k & 1);
  const bool first = k == 0;
  const v4f* r_in = reinterpret_cast<const v4f*>(rbuf + (par ? ld : 0));
  v4f* r_out = reinterpret_cast<v4f*>(rbuf + (par ? 0 : ld));
  const int nk = static_cast<int>(gridDim.x);  // <= kCorrThreads (host-checked)
  const uint64_t* k_in = keys + (par ? nk : 0);
  uint64_t* k_out = keys + (par ? 0 : nk);

  // requests first, all unconditional (clamped indices into valid memory)
  int done_v = 0;
  if (threadIdx.x == 0)
    done_v = __hip_atomic_load(&st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // eps^2 ||y||^2, set by the init kernel before the first launch
  const double thr = st->thr;
  v4f rq[RPT];
#pragma unroll
  for (int u = 0; u < RPT; ++u) {
    const int i = threadIdx.x + u * kCorrThreads;
    rq[u] = r_in[i < ld4 ? i : ld4 - 1];
  }
  uint64_t kp = k_in[static_cast<int>(threadIdx.x) < nk ? static_cast<int>(threadIdx.x) : nk - 1];
  if (first || static_cast<int>(threadIdx.x) >= nk) kp = 0;
  const unsigned dur_prev = bal->dur[par ^ 1][static_cast<int>(threadIdx.x) < nk ? threadIdx.x : 0];
  const int sh_prev = bal->share[par ^ 1][threadIdx.x % kBalGroups];
#pragma unroll
  for (int u = 0; u < RPT; ++u) {
    const int i = threadIdx.x + u * kCorrThreads;
    if (i < ld4) r_lds[i] = rq[u];
  }
  if (threadIdx.x == 0) s_done = done_v;  // one value for the whole workgroup
  __syncthreads();
  if (s_done) return;
  int64_t col0, col1;
  balanced_range<kCorrThreads>(bal, par, !first, nk, m, cols_per_wg, dur_prev, sh_prev, col0,
                               col1);

  if (!first) {
    const uint64_t win = block_max<kCorrThreads>(kp, kred);
    const int idx = key_index(win);
    const float c = key_value(win);
    if (carried_winner_stops(idx, c, m, st)) return;
    if (carried_update<kCorrThreads>(idx, c, psi, ld, n, r_lds, r_out, x, st, tr, k, max_iters, thr,
                                     par ^ 1, dred))
      return;
  } else if (blockIdx.x == 0) {
    for (int i = threadIdx.x; i < ld4; i += kCorrThreads) r_out[i] = r_lds[i];
    if (threadIdx.x == 0) st->r_sel = par ^ 1;
  }

  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const unsigned long long t_begin = wall_clock64();
  uint64_t best = 0;
  for (int64_t col = col0 + wave; col < col1; col += kCorrThreads / kWave) {
    const float c = dot_column_f32(reinterpret_cast<const v4f*>(psi + col * ld), r_lds, ld4, lane);
    const uint64_t key = make_key(c, static_cast<int>(col));
    best = key > best ? key : best;
  }
  best = block_max<kCorrThreads>(best, kred);
  if (threadIdx.x == 0) k_out[blockIdx.x] = best;
  record_pass_time(bal, par, t_begin);
}

// ---------------------------------------------------------------------------
// Small dictionaries: the whole decode in one launch of G <= kSmallMaxWgs
// workgroups (one per CU), each holding its share of the columns in LDS for
// the whole decode, so a step reads no dictionary bytes from memory.
//
// Step k does what launch k of k_mp_step_f32 does, with the same code for
// the selection (the largest key of all workgroups, eq. 16), the update
// (carried_update: every workgroup applies step k to its own LDS copy of r
// and sums ||r_k||^2 in FP64 in the same order; workgroup 0 also keeps r,
// x~, the trace and the state) and the correlations (dot_column_f32 over
// the column's LDS copy, the same FMAs in the same order as over its copy in
// memory), so results are bit-identical to the stepping form; which
// workgroup or wave scores a column does not change its correlation, and
// the largest key does not depend on the order the keys are compared in.
// In place of the kernel boundary, every wave publishes its best key of
// pass k as two 64-bit words, each a 32-bit tag (decode epoch, step) over 32
// bits of the key, with relaxed device-scope atomics, as soon as its columns
// are scored (no reduction inside the workgroup first), and every workgroup
// reads all waves' words of the pass before it goes on; steps alternate
// between two halves of the slots (a wave overwrites its words of pass k
// only after its workgroup read every record of pass k+1, each of which its
// owner published after its own workgroup read every record of pass k).
// The epoch, new for every decode, keeps words of an earlier decode from
// matching.
//
// Every wait ends: the host launches this form only where the occupancy
// query shows every workgroup resident at once (one per CU, G <= CUs), all
// workgroups take the same decisions from the same gathered keys, and a
// wait that has polled `spin_limit` times in vain sets the sticky
// DevState::fail word and leaves, after which every other workgroup's wait
// gives up too.
constexpr int kSmallLds = 150 * 1024;  // dynamic LDS for r and a share, at most
constexpr int kSmallMaxWgs = 32;
constexpr int kSmallWaves = kCorrThreads / kWave;  // records per workgroup and pass
constexpr int kSmallRecs = kSmallMaxWgs * kSmallWaves;
constexpr int kSmallCols = 8;  // columns a wave scores at once
static_assert(kSmallRecs <= kCorrThreads, "one polling thread per record");
constexpr unsigned kSmallEpochMod = 4096;

__global__ __launch_bounds__(kCorrThreads) void k_f32_small(
    const float* __restrict__ psi, int64_t ld, int64_t n, int64_t m, float* __restrict__ rbuf,
    int cols_per_wg, unsigned long long* __restrict__ slots, unsigned epoch,
    long long spin_limit, long long max_iters, float* __restrict__ x,
    DevState* __restrict__ st, mp_trace tr) {
  extern __shared__ v4f smem[];  // r (ld4 float4s), then the share's columns
  __shared__ uint64_t s_keys[kSmallRecs];  // the polled keys of a pass
  __shared__ double dred[kCorrThreads / kWave];
  __shared__ int s_flag;
  const int ld4 = static_cast<int>(ld / 4);
  const int G = static_cast<int>(gridDim.x);
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  v4f* r_lds = smem;
  v4f* cols = smem + ld4;
  const int64_t col0 = static_cast<int64_t>(blockIdx.x) * cols_per_wg;
  int64_t col1 = col0 + cols_per_wg;
  if (col1 > m) col1 = m;
  const unsigned ep = (epoch % kSmallEpochMod) << 20;

  if (threadIdx.x == 0)
    s_flag = __hip_atomic_load(&st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const double thr = st->thr;
  // r = y (half 0, written by the init kernel) and the share's columns into LDS
  const v4f* r_in = reinterpret_cast<const v4f*>(rbuf);
  for (int i = threadIdx.x; i < ld4; i += kCorrThreads) r_lds[i] = r_in[i];
  {
    const v4f* src = reinterpret_cast<const v4f*>(psi + col0 * ld);
    const int total = static_cast<int>(col1 - col0) * ld4;
    for (int i = threadIdx.x; i < total; i += kCorrThreads) cols[i] = src[i];
  }
  __syncthreads();
  if (s_flag) return;  // the init kernel stopped the run (zero or non-finite y, T = 0, ...)
  __syncthreads();     // s_flag is reused below
  if (threadIdx.x == 0) s_flag = 0;
  v4f* r_out = reinterpret_cast<v4f*>(rbuf + ld);  // workgroup 0 keeps r_k here (half 1)

  for (long long k = 0;; ++k) {
    if (k > 0) {
      // every wave's key of pass k (published with step field k): record
      // wg * kSmallWaves + wave of the pass's half
      uint64_t kp = 0;
      if (static_cast<int>(threadIdx.x) < G * kSmallWaves) {
        const unsigned want = ep | (static_cast<unsigned>(k) & 0xFFFFFu);
        unsigned long long* w0 = slots + ((k & 1) * kSmallRecs + threadIdx.x) * 2;
        long long spins = 0;
        unsigned long long hi = 0, lo = 0;
        for (;;) {
          if (spins >= spin_limit) {  // spin_limit polls have failed (0: none is made)
            s_flag = 1;
            break;
          }
          lo = __hip_atomic_load(w0 + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (static_cast<unsigned>(lo >> 32) == want) {
            hi = __hip_atomic_load(w0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (static_cast<unsigned>(hi >> 32) == want) break;
          }
          ++spins;
          __builtin_amdgcn_s_sleep(1);
        }
        kp = ((hi & 0xFFFFFFFFull) << 32) | (lo & 0xFFFFFFFFull);
        s_keys[threadIdx.x] = kp;
      }
      __syncthreads();
      if (s_flag) {
        if (threadIdx.x == 0) {
          (void)__hip_atomic_fetch_or(&st->fail, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(&st->done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        return;
      }
      // every wave takes the largest of the polled keys itself (the same in
      // all: the largest key does not depend on the order of comparison),
      // with no further barrier; s_keys is written again only after the
      // barriers of the update below
      uint64_t v = 0;
      for (int i = lane; i < G * kSmallWaves; i += kWave) v = s_keys[i] > v ? s_keys[i] : v;
      const uint64_t win = wave_max(v);
      const int idx = key_index(win);
      const float c = key_value(win);
      if (carried_winner_stops(idx, c, m, st)) return;
      if (carried_update<kCorrThreads>(idx, c, psi, ld, n, r_lds, r_out, x, st, tr, k, max_iters,
                                       thr, 1, dred))
        return;
    }
    // pass k+1 over the share, from LDS: kSmallCols of the wave's columns at
    // a time, so that their loads and lane sums overlap, each with
    // dot_column_f32's arithmetic (the two chains over the column's halves,
    // each lane's elements in increasing order, then the lane sum), then the
    // rest one by one
    uint64_t best = 0;
    int64_t col = col0 + wave;
    const int h0 = ld4 / 2;
    for (; col + kSmallWaves * (kSmallCols - 1) < col1; col += kSmallWaves * kSmallCols) {
      float acc_a[kSmallCols], acc_b[kSmallCols];
#pragma unroll
      for (int u = 0; u < kSmallCols; ++u) acc_a[u] = acc_b[u] = 0.0f;
      for (int i = lane; i < h0; i += kWave) {
        const v4f ra = r_lds[i], rb = r_lds[h0 + i];
#pragma unroll
        for (int u = 0; u < kSmallCols; ++u) {
          const v4f* p = cols + (col + kSmallWaves * u - col0) * ld4;
          const v4f a = p[i], b = p[h0 + i];
          acc_a[u] = __builtin_fmaf(a.x, ra.x, acc_a[u]);
          acc_a[u] = __builtin_fmaf(a.y, ra.y, acc_a[u]);
          acc_a[u] = __builtin_fmaf(a.z, ra.z, acc_a[u]);
          acc_a[u] = __builtin_fmaf(a.w, ra.w, acc_a[u]);
          acc_b[u] = __builtin_fmaf(b.x, rb.x, acc_b[u]);
          acc_b[u] = __builtin_fmaf(b.y, rb.y, acc_b[u]);
          acc_b[u] = __builtin_fmaf(b.z, rb.z, acc_b[u]);
          acc_b[u] = __builtin_fmaf(b.w, rb.w, acc_b[u]);
        }
      }
#pragma unroll
      for (int u = 0; u < kSmallCols; ++u) {
        const float cv = wave_sum(acc_a[u] + acc_b[u]);
        const uint64_t key = make_key(cv, static_cast<int>(col + kSmallWaves * u));
        best = key > best ? key : best;
      }
    }
    for (; col < col1; col += kSmallWaves) {
      const float cv = dot_column_f32<false>(cols + (col - col0) * ld4, r_lds, ld4, lane);
      const uint64_t key = make_key(cv, static_cast<int>(col));
      best = key > best ? key : best;
    }
    // this wave's key (the same in every lane: each correlation is the wave's
    // lane sum) published at once
    if (lane == 0) {
      const unsigned long long tag =
          static_cast<unsigned long long>(ep | (static_cast<unsigned>(k + 1) & 0xFFFFFu)) << 32;
      unsigned long long* w0 =
          slots + (((k + 1) & 1) * kSmallRecs + blockIdx.x * kSmallWaves + wave) * 2;
      __hip_atomic_store(w0, tag | (best >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(w0 + 1, tag | (best & 0xFFFFFFFFull), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// Launch shape of the small-dictionary decode for an FP32 context, or
// grid 0 where it does not apply (the share and r must fit the LDS limit,
// at most kSmallMaxWgs workgroups, all resident at once).
CorrGeom small_geometry(int64_t ld, int64_t m, int num_cus) {
  CorrGeom g{0, 0};
  constexpr int64_t kWaves = kCorrThreads / kWave;
  const int64_t room = (kSmallLds - 4 * ld) / (4 * ld);  // columns that fit beside r
  if (room < kWaves || ld > 16384) return g;
  const int64_t cap = room / kWaves * kWaves;
  int64_t grid = (m + cap - 1) / cap;
  if (grid > kSmallMaxWgs || grid > num_cus) return g;
  int64_t cpw = (m + grid - 1) / grid;
  cpw = (cpw + kWaves - 1) / kWaves * kWaves;  // a whole number of columns per wave
  grid = (m + cpw - 1) / cpw;
  static bool attr_set = false;
  if (!attr_set) {
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(k_f32_small),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kSmallLds) != hipSuccess)
      return g;
    attr_set = true;
  }
  int per_cu = 0;
  const size_t lds = static_cast<size_t>(4 * ld * (cpw + 1));
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(
                                                       k_f32_small),
                                                   kCorrThreads, lds) != hipSuccess ||
      per_cu < 1)
    return g;
  g.cols_per_wg = static_cast<int>(cpw);
  g.grid = static_cast<int>(grid);
  return g;
}

hipError_t launch_f32_small(const float* psi, int64_t ld, int64_t n, int64_t m, float* rbuf,
                            const CorrGeom& g, unsigned long long* slots, unsigned epoch,
                            long long max_iters, float* x, DevState* st, mp_trace tr,
                            hipStream_t s) {
  if (g.grid < 1 || g.grid > kSmallMaxWgs) return hipErrorInvalidValue;
  // polls per wait before the run is marked failed; MP_SMALL_SPIN_LIMIT (a
  // non-negative integer; 0 gives up at the first wait) overrides it, so
  // that tests can drive the failure path
  long long spin_limit = 1ll << 22;
  if (const char* env = getenv("MP_SMALL_SPIN_LIMIT")) {
    char* end = nullptr;
    const long long v = strtoll(env, &end, 10);
    if (end != env && v >= 0) spin_limit = v;
  }
  const size_t lds = static_cast<size_t>(4 * ld * (g.cols_per_wg + 1));
  if (lds > static_cast<size_t>(kSmallLds)) return hipErrorInvalidValue;
  k_f32_small<<<dim3(g.grid), dim3(kCorrThreads), lds, s>>>(psi, ld, n, m, rbuf, g.cols_per_wg,
                                                            slots, epoch, spin_limit, max_iters,
                                                            x, st, tr);
  return hipGetLastError();
}

unsigned small_epoch_mod() { return kSmallEpochMod; }
int small_slot_words() { return 2 * kSmallRecs * 2; }

// The first n floats of the residual half the state names (st->r_sel) into
// r: the end of a carried decode, one launch instead of a host round trip.
__global__ __launch_bounds__(256) void k_copy_selected(const float* __restrict__ rbuf, int64_t ld,
                                                       int64_t n, const DevState* __restrict__ st,
                                                       float* __restrict__ r) {
  const float* src = rbuf + (st->r_sel ? ld : 0);
  const int64_t stride = static_cast<int64_t>(gridDim.x) * 256;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < n; i += stride)
    r[i] = src[i];
}

hipError_t launch_copy_selected(const float* rbuf, int64_t ld, int64_t n, const DevState* st,
                                float* r, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 64);
  k_copy_selected<<<dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s>>>(rbuf, ld, n, st, r);
  return hipGetLastError();
}

CorrGeom corr_f32_geometry(int64_t m, int num_cus) {
  // One 16-wave workgroup per CU (one LDS copy of r per CU, few keys);
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

hipError_t launch_mp_step_f32(const float* psi, int64_t ld, int64_t n, int64_t m, float* rbuf,
                              const CorrGeom& g, uint64_t* keys, BalState* bal, long long k,
                              long long max_iters, float* x, DevState* st, mp_trace tr,
                              hipStream_t s) {
  const size_t lds = static_cast<size_t>(ld) * sizeof(float);
  static bool big_lds = false;  // residuals above 60 KB need the opt-in limit
  if (!big_lds && lds > 60 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_mp_step_f32),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
    if (e != hipSuccess) return e;
    big_lds = true;
  }
  k_mp_step_f32<<<dim3(g.grid), dim3(kCorrThreads), lds, s>>>(
      psi, ld, n, m, rbuf, g.cols_per_wg, keys, bal, k, max_iters, x, st, tr);
  return hipGetLastError();
}

}  // namespace mp
