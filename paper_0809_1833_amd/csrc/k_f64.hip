// FP64 single-signal Matching Pursuit for gfx950 (Section 3, eqs. 8-12): the
// double-precision configuration the paper times beside the single-precision
// one (Section 4).  Dictionary, y, x~, r and every inner product are FP64.
//
// The launch structure is the FP32 form's: one MP iteration per launch, one
// 16-wave workgroup per CU, r staged whole in LDS (N <= 16384 doubles =
// 128 KB), each column streamed with 16-byte non-temporal loads (two doubles)
// and summed with FP64 FMAs in two per-lane chains over the column halves,
// then across the wave.  A candidate is a pair of 64-bit words so that the
// exact FP64 coefficient survives the argmax: the |c| bits (a non-negative
// double orders like its bit pattern), then (0x7FFFFFFF - index) and the
// sign; the pair order is "larger |c|, then smaller index" (eq. 16).  The
// selection is carried into the next launch, where every workgroup takes the
// winner from the stored pairs, updates its copy of r and applies the FP64
// stopping test.
#include "k_common.h"
#include "k_key2.h"
#include "mp_internal.h"

namespace mp {

typedef double v2d __attribute__((ext_vector_type(2)));

constexpr int kF64Threads = 1024;
constexpr int kF64Waves = kF64Threads / kWave;

// ---- FP64 inner product of one column with the LDS copy of r -----------------
//
// Lane l sums the 16-byte chunks (two doubles) l, l+64, ... below h0 = ld2/2
// into one FP64 accumulator and h0+l, h0+l+64, ... into another, each in
// increasing order with FMAs; the two are added per lane and the wave sums
// the lanes.

template <int U>
__device__ inline void dot_block2_f64(const v2d* __restrict__ p, const v2d* __restrict__ r_lds,
                                      int h0, int& i, double& acc_a, double& acc_b) {
  v2d a[U], b[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    a[u] = __builtin_nontemporal_load(p + i + kWave * u);
    b[u] = __builtin_nontemporal_load(p + h0 + i + kWave * u);
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const v2d ra = r_lds[i + kWave * u];
    acc_a = __builtin_fma(a[u].x, ra.x, acc_a);
    acc_a = __builtin_fma(a[u].y, ra.y, acc_a);
    const v2d rb = r_lds[h0 + i + kWave * u];
    acc_b = __builtin_fma(b[u].x, rb.x, acc_b);
    acc_b = __builtin_fma(b[u].y, rb.y, acc_b);
  }
  i += kWave * U;
}

__device__ inline double dot_column_f64(const v2d* __restrict__ p, const v2d* __restrict__ r_lds,
                                        int ld2, int lane) {
  const int h0 = ld2 / 2;
  double acc_a = 0.0, acc_b = 0.0;
  int i = lane;
  while (i + kWave * 7 < h0) dot_block2_f64<8>(p, r_lds, h0, i, acc_a, acc_b);
  if (i + kWave * 3 < h0) dot_block2_f64<4>(p, r_lds, h0, i, acc_a, acc_b);
  if (i + kWave * 1 < h0) dot_block2_f64<2>(p, r_lds, h0, i, acc_a, acc_b);
  if (i < h0) dot_block2_f64<1>(p, r_lds, h0, i, acc_a, acc_b);
  return wave_sum(acc_a + acc_b);
}

// ---------------------------------------------------------------------------
// Set-up check of eq. 4: norm2[m] = sum_n psi_nm^2 in FP64, one wave per column.
__global__ __launch_bounds__(256) void k_norms_f64(const double* __restrict__ psi, int64_t ld,
                                                   int64_t n, int64_t m,
                                                   double* __restrict__ norm2) {
  const int lane = threadIdx.x % kWave;
  const int64_t col = static_cast<int64_t>(blockIdx.x) * 4 + threadIdx.x / kWave;
  if (col >= m) return;
  const double* p = psi + col * ld;
  double s = 0.0;
  for (int64_t i = lane; i < n; i += kWave) s = __builtin_fma(p[i], p[i], s);
  s = wave_sum(s);
  if (lane == 0) norm2[col] = s;
}

// Init (eq. 8): r = y (zero padded to ld), x~ = 0, t = 0, ||y||^2, pre-test.
__global__ __launch_bounds__(256) void k_init_f64(const double* __restrict__ y, int64_t n,
                                                  int64_t ld, double* __restrict__ x, int64_t m,
                                                  double* __restrict__ r,
                                                  DevState* __restrict__ st, double eps,
                                                  long long max_iters) {
  __shared__ double red[4];
  const int64_t gtid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t gstride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t j = gtid; j < m; j += gstride) x[j] = 0.0;
  if (blockIdx.x != 0) return;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < ld; i += 256) {
    const double v = i < n ? y[i] : 0.0;
    r[i] = v;
    s = __builtin_fma(v, v, s);
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

// ---------------------------------------------------------------------------
// One MP step per launch (eqs. 9-12), the selection carried into the next
// launch as in the FP32 form.  Launch k (k >= 1): every workgroup stages
// r_{k-1} (half k mod 2 of the residual buffer) in LDS and reads the pairs
// the workgroups of launch k-1 stored; all take the same winner, apply step
// k to their LDS copy (r -= c psi_idx, FP64 FMAs) and reduce ||r_k||^2 in the
// same order, so all reach the same stop decision; workgroup 0 stores r_k in
// the other half and keeps x~, the trace and the state.  Unless the run
// stops, each runs pass k+1 over its share of the columns (balanced between
// the XCDs from the previous launch's pass times, as in the FP32 form) and
// stores its best pair.  Launch 0 runs the first pass on r = y; T steps take
// T+1 launches.
__global__ __launch_bounds__(kF64Threads) void k_mp_step_f64(
    const double* __restrict__ psi, int64_t ld, int64_t n, int64_t m, double* __restrict__ rbuf,
    int cols_per_wg, uint64_t* __restrict__ keys, BalState* __restrict__ bal, long long k,
    long long max_iters, double thr, double* __restrict__ x, DevState* __restrict__ st,
    mp_trace_f64 tr) {
  extern __shared__ v2d r2_lds[];
  __shared__ Key2 kred[kF64Waves];
  __shared__ double dred[kF64Waves];
  __shared__ int s_done;
  constexpr int RPT = 16384 / 2 / kF64Threads;  // 16-byte chunks of r per thread (ld <= 16384)
  const int ld2 = static_cast<int>(ld / 2);
  const int par = static_cast<int>(k & 1);
  const bool first = k == 0;
  const v2d* r_in = reinterpret_cast<const v2d*>(rbuf + (par ? ld : 0));
  v2d* r_out = reinterpret_cast<v2d*>(rbuf + (par ? 0 : ld));
  const int nk = static_cast<int>(gridDim.x);  // <= kF64Threads (host-checked)
  const uint64_t* k_in = keys + (par ? 2 * nk : 0);
  uint64_t* k_out = keys + (par ? 0 : 2 * nk);
  const int t = static_cast<int>(threadIdx.x);

  // requests first, all unconditional (clamped indices into valid memory)
  int done_v = 0;
  if (t == 0) done_v = __hip_atomic_load(&st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  v2d rq[RPT];
#pragma unroll
  for (int u = 0; u < RPT; ++u) {
    const int i = t + u * kF64Threads;
    rq[u] = r_in[i < ld2 ? i : ld2 - 1];
  }
  const int tc = t < nk ? t : nk - 1;
  Key2 kp{k_in[2 * tc], k_in[2 * tc + 1]};
  if (first || t >= nk) kp = Key2{0, 0};
  const unsigned dur_prev = bal->dur[par ^ 1][tc];
  const int sh_prev = bal->share[par ^ 1][t % kBalGroups];
#pragma unroll
  for (int u = 0; u < RPT; ++u) {
    const int i = t + u * kF64Threads;
    if (i < ld2) r2_lds[i] = rq[u];
  }
  if (t == 0) s_done = done_v;  // one value for the whole workgroup
  __syncthreads();
  if (s_done) return;
  int64_t col0, col1;
  balanced_range<kF64Threads>(bal, par, !first, nk, m, cols_per_wg, dur_prev, sh_prev, col0,
                              col1);

  if (!first) {
    const Key2 w = block_max_key2<kF64Threads>(kp, kred);
    const int idx = key2_index(w);
    const double c = key2_value(w);
    const bool bad = w.lo == 0 || idx < 0 || idx >= m;  // no published pair is
    if (bad || c == 0.0) {  // c = 0: no atom correlates with r
      if (blockIdx.x == 0 && t == 0) {
        st->reason = bad ? kStopInternal : MP_STOP_STALLED;
        st->done = 1;
      }
      return;
    }
    // r <- r - c psi_idx on the LDS copy, all column loads first; padding
    // rows stay +0
    const v2d* colp = reinterpret_cast<const v2d*>(psi + static_cast<int64_t>(idx) * ld);
    v2d a[RPT];
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      const int i = t + u * kF64Threads;
      a[u] = colp[i < ld2 ? i : ld2 - 1];
    }
    // workgroup 0: this step's residual trace entry, if the trace asks for one
    double* rt = blockIdx.x == 0 && tr.r && k - 1 < tr.cap ? tr.r + (k - 1) * tr.ldr : nullptr;
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      const int i = t + u * kF64Threads;
      if (i < ld2) {
        const v2d rv = r2_lds[i];
        v2d o;
        o.x = __builtin_fma(-c, a[u].x, rv.x);
        o.y = __builtin_fma(-c, a[u].y, rv.y);
        r2_lds[i] = o;
        if (blockIdx.x == 0) r_out[i] = o;
        if (rt) {
          if (2 * i < n) rt[2 * i] = o.x;
          if (2 * i + 1 < n) rt[2 * i + 1] = o.y;
        }
        s = __builtin_fma(o.x, o.x, s);
        s = __builtin_fma(o.y, o.y, s);
      }
    }
    const double rr = block_sum<kF64Threads>(s, dred);  // its barriers order the LDS writes
    if (blockIdx.x == 0 && t == 0) {
      x[idx] += c;
      const long long tt = k - 1;
      if (tt < tr.cap) {
        if (tr.idx) tr.idx[tt] = idx;
        if (tr.coef) tr.coef[tt] = c;
        if (tr.rr) tr.rr[tt] = rr;
      }
      st->t = k;
      st->rr = rr;
      st->r_sel = par ^ 1;
      if (!(rr > thr)) {
        st->reason = MP_STOP_CONVERGED;
        st->done = 1;
      } else if (k >= max_iters) {
        st->reason = MP_STOP_MAX_ITERS;
        st->done = 1;
      }
    }
    if (!(rr > thr) || k >= max_iters) return;
  } else if (blockIdx.x == 0) {
    for (int i = t; i < ld2; i += kF64Threads) r_out[i] = r2_lds[i];
    if (t == 0) st->r_sel = par ^ 1;
  }

  const int lane = t % kWave, wave = t / kWave;
  const unsigned long long t_begin = wall_clock64();
  Key2 best{0, 0};
  for (int64_t col = col0 + wave; col < col1; col += kF64Waves) {
    const double c =
        dot_column_f64(reinterpret_cast<const v2d*>(psi + col * ld), r2_lds, ld2, lane);
    best = key2_max(best, make_key2(c, static_cast<int>(col)));
  }
  best = block_max_key2<kF64Threads>(best, kred);
  if (t == 0) k_out[2 * blockIdx.x] = best.hi;
  if (t == 1) k_out[2 * blockIdx.x + 1] = best.lo;
  record_pass_time(bal, par, t_begin);
}

// ---------------------------------------------------------------------------

hipError_t launch_norms_f64(const double* psi, int64_t ld, int64_t n, int64_t m, double* norm2,
                            hipStream_t s) {
  const int64_t blocks = (m + 3) / 4;
  k_norms_f64<<<dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s>>>(psi, ld, n, m, norm2);
  return hipGetLastError();
}

hipError_t launch_init_f64(const double* y, int64_t n, int64_t ld, double* x, int64_t m,
                           double* r, DevState* st, double eps, long long max_iters,
                           hipStream_t s) {
  int64_t blocks = (m + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  k_init_f64<<<dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s>>>(y, n, ld, x, m, r, st,
                                                                        eps, max_iters);
  return hipGetLastError();
}

hipError_t launch_mp_step_f64(const double* psi, int64_t ld, int64_t n, int64_t m, double* rbuf,
                              const CorrGeom& g, uint64_t* keys, BalState* bal, long long k,
                              long long max_iters, double thr, double* x, DevState* st,
                              mp_trace_f64 tr, hipStream_t s) {
  const size_t lds = static_cast<size_t>(ld) * sizeof(double);
  static size_t lds_set = 60 * 1024;  // above the default limit the opt-in is raised
  if (lds > lds_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_mp_step_f64),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(lds));
    if (e != hipSuccess) return e;
    lds_set = lds;
  }
  k_mp_step_f64<<<dim3(g.grid), dim3(kF64Threads), lds, s>>>(
      psi, ld, n, m, rbuf, g.cols_per_wg, keys, bal, k, max_iters, thr, x, st, tr);
  return hipGetLastError();
}

}  // namespace mp
