// FP32 single-signal Matching Pursuit kernels for gfx950 (Section 3, eqs. 8-12).
//
// One MP iteration is two launches on the caller's stream:
//   corr_f32           c_m = <r, psi_m> for every column (eq. 9), streaming the
//                      whole column-major dictionary once; each workgroup
//                      keeps its best |c_m| (smallest index on ties, eq. 16)
//                      and writes one packed key.
//   select_update_f32  one workgroup: the best of those keys picks i; then
//                      x~_i += c_i (eq. 10), r -= c_i psi_i (eq. 11), t += 1
//                      (eq. 12), ||r||^2 in FP64 and the stopping test.
// Both return at once when the device state says the run has stopped, so the
// host can enqueue iterations ahead without reading anything back.
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
// Correlation pass (eq. 9) with a fused per-workgroup argmax.
//
// Workgroup = 4 waves.  The residual (ld floats, zero padded) is staged once
// into LDS; wave w of workgroup b takes columns b*cpw + w, + 4, ... and
// streams each column with 16-byte non-temporal loads (lane l reads float4s
// l, l+64, ...), UNROLL loads in flight per lane, FP32 FMA accumulation,
// then a butterfly sum across the wave.  Keys are max-reduced per wave and
// then across the 4 waves; one key per workgroup goes to `partials`.
constexpr int kCorrThreads = 256;
constexpr int kCorrUnroll = 8;

__global__ __launch_bounds__(kCorrThreads) void k_corr_f32(const float* __restrict__ psi,
                                                           int64_t ld, int64_t m,
                                                           const float* __restrict__ r,
                                                           int cols_per_wg,
                                                           uint64_t* __restrict__ partials,
                                                           const DevState* __restrict__ st) {
  if (st->done) return;
  extern __shared__ v4f r_lds[];
  __shared__ uint64_t red[kCorrThreads / kWave];
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
    const v4f* p = reinterpret_cast<const v4f*>(psi + col * ld);
    float acc = 0.0f;
    int i = lane;
    for (; i + kWave * (kCorrUnroll - 1) < ld4; i += kWave * kCorrUnroll) {
      v4f a[kCorrUnroll];
#pragma unroll
      for (int u = 0; u < kCorrUnroll; ++u) a[u] = __builtin_nontemporal_load(p + i + kWave * u);
#pragma unroll
      for (int u = 0; u < kCorrUnroll; ++u) {
        const v4f b = r_lds[i + kWave * u];
        acc = __builtin_fmaf(a[u].x, b.x, acc);
        acc = __builtin_fmaf(a[u].y, b.y, acc);
        acc = __builtin_fmaf(a[u].z, b.z, acc);
        acc = __builtin_fmaf(a[u].w, b.w, acc);
      }
    }
    for (; i < ld4; i += kWave) {
      const v4f a = __builtin_nontemporal_load(p + i);
      const v4f b = r_lds[i];
      acc = __builtin_fmaf(a.x, b.x, acc);
      acc = __builtin_fmaf(a.y, b.y, acc);
      acc = __builtin_fmaf(a.z, b.z, acc);
      acc = __builtin_fmaf(a.w, b.w, acc);
    }
    acc = wave_sum(acc);
    const uint64_t k = make_key(acc, static_cast<int>(col));
    best = k > best ? k : best;
  }
  best = block_max<kCorrThreads>(best, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = best;
}

CorrGeom corr_f32_geometry(int64_t m, int num_cus) {
  // Aim for about four workgroups per CU; a workgroup takes at least one
  // column per wave.
  const int64_t target = static_cast<int64_t>(num_cus > 0 ? num_cus : 256) * 4;
  int64_t cpw = (m + target - 1) / target;
  cpw = ((cpw + 3) / 4) * 4;
  if (cpw < 4) cpw = 4;
  CorrGeom g;
  g.cols_per_wg = static_cast<int>(cpw);
  g.grid = static_cast<int>((m + cpw - 1) / cpw);
  return g;
}

hipError_t launch_corr_f32(const float* psi, int64_t ld, int64_t m, const float* r,
                           const CorrGeom& g, uint64_t* partials, const DevState* st,
                           hipStream_t s) {
  const size_t lds = static_cast<size_t>(ld) * sizeof(float);
  static bool big_lds = false;  // residuals above 60 KB need the opt-in limit
  if (!big_lds && lds > 60 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_corr_f32),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
    if (e != hipSuccess) return e;
    big_lds = true;
  }
  k_corr_f32<<<dim3(g.grid), dim3(kCorrThreads), lds, s>>>(psi, ld, m, r, g.cols_per_wg,
                                                           partials, st);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Select and update (eqs. 9-12 after the correlation pass), one workgroup.
constexpr int kSelThreads = 1024;

__global__ __launch_bounds__(kSelThreads) void k_select_update_f32(
    const uint64_t* __restrict__ partials, int np, const float* __restrict__ psi, int64_t ld,
    int64_t n, float* __restrict__ x, float* __restrict__ r, DevState* __restrict__ st,
    mp_trace tr) {
  __shared__ uint64_t kred[kSelThreads / kWave];
  __shared__ double dred[kSelThreads / kWave];
  if (st->done) return;
  uint64_t best = 0;
  for (int i = threadIdx.x; i < np; i += kSelThreads) {
    const uint64_t k = partials[i];
    best = k > best ? k : best;
  }
  best = block_max<kSelThreads>(best, kred);
  const int idx = key_index(best);
  const float c = key_value(best);
  if (c == 0.0f) {  // no atom correlates with r: MP cannot make progress
    if (threadIdx.x == 0) {
      st->done = 1;
      st->reason = MP_STOP_STALLED;
    }
    return;
  }
  const float* col = psi + static_cast<int64_t>(idx) * ld;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kSelThreads) {
    const float v = __builtin_fmaf(-c, col[i], r[i]);
    r[i] = v;
    s += static_cast<double>(v) * v;
  }
  const double rr = block_sum<kSelThreads>(s, dred);
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

hipError_t launch_select_update_f32(const uint64_t* partials, int np, const float* psi,
                                    int64_t ld, int64_t n, float* x, float* r, DevState* st,
                                    mp_trace tr, hipStream_t s) {
  k_select_update_f32<<<dim3(1), dim3(kSelThreads), 0, s>>>(partials, np, psi, ld, n, x, r, st,
                                                            tr);
  return hipGetLastError();
}

}  // namespace mp
