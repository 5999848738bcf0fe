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
// across the 16 waves; each workgroup publishes its key and counts itself in
// (publish_arrive).  The workgroup that arrives last (nobody waits: it is
// simply the one that sees the count reach the grid size) takes the winning
// key, updates x~ and r, computes ||r||^2 in FP64 and applies the stopping
// test.
constexpr int kCorrThreads = 1024;

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
  if (!publish_arrive<1>(best, keys, st)) return;
  // last workgroup: the launch's winner is the largest published key
  uint64_t winner = 0;
  for (int i = threadIdx.x; i < static_cast<int>(gridDim.x); i += kCorrThreads) {
    const uint64_t k = take_slot(keys + i);
    winner = k > winner ? k : winner;
  }
  winner = block_max<kCorrThreads>(winner, kred);
  select_update_tail<kCorrThreads>(winner, psi, ld, n, m, x, r, r_lds, st, tr, dred);
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
