// Orthogonal Matching Pursuit for gfx950, FP32 (the refinement of MP the
// paper names as its next target): MP's selection (eq. 9 with the tie rule of
// eq. 16), then all selected atoms re-fitted by least squares so that r stays
// orthogonal to them.
//
// The least-squares fit is kept as a QR factorisation of the selected atoms,
// Psi_S = Q R, grown by one column per iteration:
//   select  i = argmax |<r, psi_m>|             (the correlation pass)
//   project w = psi_i - Q (Q^T psi_i), twice     (classical Gram-Schmidt run
//           two times: the second pass removes what rounding left of the
//           first, keeping Q orthonormal to FP32 accuracy)
//   update  rho = ||w||, q_t = w / rho, R[:t, t] = h_1 + h_2, R[t, t] = rho,
//           z_t = <q_t, r>, r -= z_t q_t, FP64 ||r||^2 and the stop test
//   finally x_S = R^-1 z (back substitution in FP64), scattered into x~.
// Each stage is its own launch; all of them return at once when the device
// state says the run is over, so the host can enqueue iterations ahead.
#include "k_common.h"
#include "mp_internal.h"

namespace mp {

constexpr int kOmpThreads = 1024;
constexpr int kOmpWaves = kOmpThreads / kWave;
constexpr int kOrthRows = 64;                  // rows of w per workgroup of k_omp_orth
constexpr int kOrthWaves = 16;                 // the sum over j split 16 ways
constexpr int kOrthThreads = kOrthWaves * kWave;
constexpr int kProjSliceMax = 16384 / 4 / kOmpProjSlices;  // float4s of a slice (ld <= 16384)

// ---------------------------------------------------------------------------
// Selection: the FP32 correlation pass and argmax of the MP step; the last
// workgroup records the selected atom (no update of x~ or r here).
__global__ __launch_bounds__(kOmpThreads) void k_omp_select(
    const float* __restrict__ psi, int64_t ld, int64_t m, const float* __restrict__ r,
    int cols_per_wg, uint64_t* __restrict__ keys, DevState* __restrict__ st,
    OmpState* __restrict__ os, unsigned char* __restrict__ in_s, int* __restrict__ sel) {
  if (st->done) return;
  extern __shared__ v4f r_lds[];
  __shared__ uint64_t kred[kOmpWaves];
  const int ld4 = static_cast<int>(ld / 4);
  const v4f* r4 = reinterpret_cast<const v4f*>(r);
  for (int i = threadIdx.x; i < ld4; i += kOmpThreads) r_lds[i] = r4[i];
  __syncthreads();
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int64_t col0 = static_cast<int64_t>(blockIdx.x) * cols_per_wg;
  int64_t col1 = col0 + cols_per_wg;
  if (col1 > m) col1 = m;
  uint64_t best = 0;
  for (int64_t col = col0 + wave; col < col1; col += kOmpWaves) {
    const float c = dot_column_f32(reinterpret_cast<const v4f*>(psi + col * ld), r_lds, ld4, lane);
    const uint64_t k = make_key(c, static_cast<int>(col));
    best = k > best ? k : best;
  }
  best = block_max<kOmpThreads>(best, kred);
  if (!publish_arrive<1>(best, keys, st)) return;
  uint64_t w = 0;
  for (int i = threadIdx.x; i < static_cast<int>(gridDim.x); i += kOmpThreads) {
    const uint64_t k = take_slot(keys + i);
    w = k > w ? k : w;
  }
  w = block_max<kOmpThreads>(w, kred);
  if (threadIdx.x == 0) {
    const int idx = key_index(w);
    const float c = key_value(w);
    if (w == 0 || idx < 0 || idx >= m) {
      st->done = 1;
      st->reason = kStopInternal;
    } else if (c == 0.0f || in_s[idx]) {  // nothing correlates, or an atom already fitted
      st->done = 1;
      st->reason = MP_STOP_STALLED;
    } else {
      const long long t = st->t;
      os->sel = idx;
      os->c = c;
      sel[t] = idx;
      in_s[idx] = 1;
    }
  }
}

// ---------------------------------------------------------------------------
// The projections <q_j, v>, j < t, by slice of rows: workgroup (b, s) stages
// slice s of v (ld / kOmpProjSlices rows) in LDS and its wave w stores
// hp[j * kOmpProjSlices + s] = sum over the slice of q_j[n] v[n] for
// j = 16 b + w (lane l sums float4s l, l + 64, ... of the slice in order,
// then the wave sums the lanes).  v is the selected atom (pass 1) or the
// partly orthogonalised w (pass 2); Q is read with caching (the next stage
// reads it again).
__global__ __launch_bounds__(kOmpThreads) void k_omp_proj(
    const float* __restrict__ q, int64_t ld, const float* __restrict__ psi,
    const float* __restrict__ wv, bool from_atom, float* __restrict__ hp,
    const DevState* __restrict__ st, const OmpState* __restrict__ os) {
  if (st->done) return;
  const long long t = st->t;
  const int64_t j0 = static_cast<int64_t>(blockIdx.x) * kOmpWaves;
  if (j0 >= t) return;  // workgroup-uniform
  __shared__ v4f v_lds[kProjSliceMax];
  const int len4 = static_cast<int>(ld / 4) / kOmpProjSlices;  // ld is a multiple of 64
  const int base = static_cast<int>(blockIdx.y) * len4;
  const float* v = from_atom ? psi + static_cast<int64_t>(os->sel) * ld : wv;
  const v4f* v4 = reinterpret_cast<const v4f*>(v) + base;
  for (int i = threadIdx.x; i < len4; i += kOmpThreads) v_lds[i] = v4[i];
  __syncthreads();
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int64_t j = j0 + wave;
  if (j < t) {
    const v4f* qj = reinterpret_cast<const v4f*>(q + j * ld) + base;
    float acc = 0.0f;
#pragma unroll 4
    for (int i = lane; i < len4; i += kWave) {
      const v4f a = qj[i], c = v_lds[i];
      acc = __builtin_fmaf(a.x, c.x, acc);
      acc = __builtin_fmaf(a.y, c.y, acc);
      acc = __builtin_fmaf(a.z, c.z, acc);
      acc = __builtin_fmaf(a.w, c.w, acc);
    }
    const float d = wave_sum(acc);
    if (lane == 0) hp[j * kOmpProjSlices + blockIdx.y] = d;
  }
}

// w[n] = v[n] - sum_{j<t} h[j] q_j[n] for the workgroup's 64 rows, with
// h[j] = the sum of j's slice projections (slices in order, staged in LDS;
// workgroup 0 also stores h for R's column): wave w sums j = w mod 16 in
// increasing order, one row per lane; the 16 partial sums are added in a
// fixed tree; the workgroup's FP64 sum of w^2 goes to part[b].
__global__ __launch_bounds__(kOrthThreads) void k_omp_orth(
    const float* __restrict__ q, int64_t ld, const float* __restrict__ psi,
    const float* __restrict__ wv_in, bool from_atom, const float* __restrict__ hp,
    float* __restrict__ h_out, float* __restrict__ w_out, double* __restrict__ part,
    const DevState* __restrict__ st, const OmpState* __restrict__ os) {
  if (st->done) return;
  extern __shared__ float h_lds[];  // t floats
  __shared__ float ps[kOrthWaves][kOrthRows];
  __shared__ double red[1];
  const long long t = st->t;
  for (long long j = threadIdx.x; j < t; j += kOrthThreads) {
    float hs = 0.0f;
#pragma unroll
    for (int s = 0; s < kOmpProjSlices; ++s) hs += hp[j * kOmpProjSlices + s];
    h_lds[j] = hs;
    if (blockIdx.x == 0) h_out[j] = hs;
  }
  __syncthreads();
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int64_t nrow = static_cast<int64_t>(blockIdx.x) * kOrthRows + lane;
  float acc = 0.0f;
#pragma unroll 4
  for (long long j = wave; j < t; j += kOrthWaves)
    acc = __builtin_fmaf(h_lds[j], q[j * ld + nrow], acc);
  ps[wave][lane] = acc;
  __syncthreads();
  if (wave == 0) {
    float p8[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) p8[k] = ps[k][lane] + ps[k + 8][lane];
    const float s = ((p8[0] + p8[4]) + (p8[2] + p8[6])) + ((p8[1] + p8[5]) + (p8[3] + p8[7]));
    const float* v = from_atom ? psi + static_cast<int64_t>(os->sel) * ld : wv_in;
    const float wn = v[nrow] - s;
    w_out[nrow] = wn;
    const double sq = wave_sum(static_cast<double>(wn) * wn);
    if (lane == 0) red[0] = sq;
  }
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// ---------------------------------------------------------------------------
// One workgroup: the new orthonormal direction, R's new column, the residual
// update and the FP64 stopping test.
__global__ __launch_bounds__(kOmpThreads) void k_omp_update(
    float* __restrict__ q, int64_t ld, int64_t n, int64_t tq, const float* __restrict__ w,
    const float* __restrict__ h1, const float* __restrict__ h2, const double* __restrict__ part,
    int nparts, float* __restrict__ rmat, double* __restrict__ z, float* __restrict__ r,
    DevState* __restrict__ st, const OmpState* __restrict__ os, mp_trace tr) {
  if (st->done) return;
  __shared__ double dred[kOmpWaves];
  const long long t = st->t;
  // w and r in registers for the whole kernel (thread i holds elements
  // i, i + kOmpThreads, ...: the order of every sum below), requested before
  // the first reduction
  constexpr int P = 16384 / kOmpThreads;  // ld <= 16384
  float wv[P], rv[P];
#pragma unroll
  for (int u = 0; u < P; ++u) {
    const int64_t i = threadIdx.x + static_cast<int64_t>(u) * kOmpThreads;
    wv[u] = i < ld ? w[i] : 0.0f;
    rv[u] = i < ld ? r[i] : 0.0f;
  }
  double s = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kOmpThreads) s += part[i];
  const double rho2 = block_sum<kOmpThreads>(s, dred);
  // the atom is (to FP32 accuracy) a combination of the atoms already fitted
  if (!(rho2 > 1e-10)) {
    if (threadIdx.x == 0) {
      st->done = 1;
      st->reason = MP_STOP_STALLED;
    }
    return;
  }
  const double rho = __builtin_sqrt(rho2);
  const float inv = static_cast<float>(1.0 / rho);
  float* qt = q + t * ld;
  double zs = 0.0;
#pragma unroll
  for (int u = 0; u < P; ++u) {
    const int64_t i = threadIdx.x + static_cast<int64_t>(u) * kOmpThreads;
    if (i < ld) {
      const float qi = wv[u] * inv;
      qt[i] = qi;
      zs += static_cast<double>(qi) * rv[u];
      wv[u] = qi;
    }
  }
  for (int64_t j = threadIdx.x; j < t; j += kOmpThreads) rmat[j + t * tq] = h1[j] + h2[j];
  const double zt = block_sum<kOmpThreads>(zs, dred);
  const float zf = static_cast<float>(zt);
  float* rt = tr.r && t < tr.cap ? tr.r + t * tr.ldr : nullptr;  // residual trace entry
  double rs = 0.0;
#pragma unroll
  for (int u = 0; u < P; ++u) {
    const int64_t i = threadIdx.x + static_cast<int64_t>(u) * kOmpThreads;
    if (i < ld) {
      const float v = __builtin_fmaf(-zf, wv[u], rv[u]);
      r[i] = v;
      if (rt && i < n) rt[i] = v;
      rs += static_cast<double>(v) * v;
    }
  }
  const double rr = block_sum<kOmpThreads>(rs, dred);
  if (threadIdx.x == 0) {
    rmat[t + t * tq] = static_cast<float>(rho);
    z[t] = zt;
    if (t < tr.cap) {
      if (tr.idx) tr.idx[t] = os->sel;
      if (tr.coef) tr.coef[t] = os->c;
      if (tr.rr) tr.rr[t] = rr;
    }
    st->t = t + 1;
    st->rr = rr;
    if (!(rr > st->thr)) {
      st->done = 1;
      st->reason = MP_STOP_CONVERGED;
    } else if (t + 1 >= st->max_iters || t + 1 >= tq) {
      st->done = 1;
      st->reason = MP_STOP_MAX_ITERS;
    }
  }
}

// x_S = R^-1 z by back substitution in FP64 (column-oriented: x_j from the
// diagonal, then z_i -= x_j R[i, j] for i < j in parallel); x~[sel[j]] = x_j.
// One workgroup; z is staged in LDS (t <= kOmpMaxT).
__global__ __launch_bounds__(kOmpThreads) void k_omp_solve(
    const float* __restrict__ rmat, int64_t tq, const double* __restrict__ z,
    const int* __restrict__ sel, const DevState* __restrict__ st, float* __restrict__ x) {
  extern __shared__ double zz[];
  __shared__ double xj_s;
  const long long t = st->t;
  for (long long i = threadIdx.x; i < t; i += kOmpThreads) zz[i] = z[i];
  __syncthreads();
  for (long long j = t - 1; j >= 0; --j) {
    if (threadIdx.x == 0) {
      const double xj = zz[j] / static_cast<double>(rmat[j + j * tq]);
      xj_s = xj;
      x[sel[j]] = static_cast<float>(xj);
    }
    __syncthreads();
    const double xj = xj_s;
    for (long long i = threadIdx.x; i < j; i += kOmpThreads)
      zz[i] -= xj * static_cast<double>(rmat[i + j * tq]);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------

hipError_t launch_omp_iteration(const float* psi, int64_t ld, int64_t n, int64_t m, float* r,
                                const CorrGeom& g, uint64_t* keys, DevState* st, OmpBufs& b,
                                long long t_bound, mp_trace tr, hipStream_t s, hipEvent_t e0,
                                hipEvent_t e1) {
  const size_t lds = static_cast<size_t>(ld) * sizeof(float);
  static bool big_lds = false;
  hipError_t e;
  if (!big_lds && lds > 60 * 1024) {
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_omp_select),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
    if (e != hipSuccess) return e;
    big_lds = true;
  }
  if (e0 && (e = hipEventRecord(e0, s)) != hipSuccess) return e;
  k_omp_select<<<dim3(g.grid), dim3(kOmpThreads), lds, s>>>(psi, ld, m, r, g.cols_per_wg, keys, st,
                                                            b.os, b.in_s, b.sel);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (e1 && (e = hipEventRecord(e1, s)) != hipSuccess) return e;
  // t <= t_bound (one more atom per iteration at most)
  const unsigned pgrid = static_cast<unsigned>(t_bound > 0 ? (t_bound + kOmpWaves - 1) / kOmpWaves : 1);
  const unsigned ogrid = static_cast<unsigned>(ld / kOrthRows);
  // h staged in LDS: tq <= 16384 floats, beside 4 KB of static LDS
  const size_t h_lds = static_cast<size_t>(b.tq) * sizeof(float);
  static bool orth_big_lds = false;
  if (!orth_big_lds && h_lds > 56 * 1024) {
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_omp_orth),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 80 * 1024);
    if (e != hipSuccess) return e;
    orth_big_lds = true;
  }
  if (ld % (4 * kOmpProjSlices) != 0 || ld / 4 / kOmpProjSlices > kProjSliceMax)
    return hipErrorInvalidValue;
  for (int pass = 0; pass < 2; ++pass) {
    const bool from_atom = pass == 0;
    float* h = pass == 0 ? b.h1 : b.h2;
    k_omp_proj<<<dim3(pgrid, kOmpProjSlices), dim3(kOmpThreads), 0, s>>>(b.q, ld, psi, b.w,
                                                                       from_atom, b.hp, st, b.os);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_omp_orth<<<dim3(ogrid), dim3(kOrthThreads), h_lds, s>>>(b.q, ld, psi, b.w, from_atom, b.hp,
                                                             h, b.w, b.part, st, b.os);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  k_omp_update<<<dim3(1), dim3(kOmpThreads), 0, s>>>(b.q, ld, n, b.tq, b.w, b.h1, b.h2, b.part,
                                                     static_cast<int>(ogrid), b.rmat, b.z, r, st,
                                                     b.os, tr);
  return hipGetLastError();
}

hipError_t launch_omp_solve(const OmpBufs& b, const DevState* st, float* x, hipStream_t s) {
  const size_t lds = static_cast<size_t>(b.tq) * sizeof(double);
  static size_t lds_set = 60 * 1024;
  if (lds > lds_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_omp_solve),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(lds));
    if (e != hipSuccess) return e;
    lds_set = lds;
  }
  k_omp_solve<<<dim3(1), dim3(kOmpThreads), lds, s>>>(b.rmat, b.tq, b.z, b.sel, st, x);
  return hipGetLastError();
}

}  // namespace mp
