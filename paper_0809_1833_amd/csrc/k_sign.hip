// Matching Pursuit on the Bernoulli dictionary of eq. 13 held as one sign bit
// per entry, for gfx950.
//
// psi_nm = (1 - 2 b_nm) / sqrt(N), so the inner product of two columns is an
// integer over N: <psi_i, psi_m> = (N - 2 popcount(b_i XOR b_m)) / N.  The
// correlations are therefore carried from step to step instead of being
// recomputed from r: with r_k = r_{k-1} - c* psi_idx (eq. 11), eq. 9 gives
//   c_m(k) = <r_k, psi_m> = c_m(k-1) - c* <psi_idx, psi_m>,
// one XOR and one bit count per 32 rows, the Gram entry exact.  The carried
// correlations and r are FP64 (after t steps the carried c stays within about
// t 2^-53 |y| of a recomputation); c(0) = Psi^T y is computed once per
// decode, in FP64, by k_sign_c0.  A pass reads N/8 bytes per column.
//
// Storage: column m is ws words at m ws (ws = ceil(N/32) rounded up to a
// multiple of 4); bit q of word w is row 32 w + q; bits of rows >= N are
// zero.  The wave that handles a column reads it in 16-byte chunks, lane l
// taking chunks l, l + 64, ... (CPL of them), and reads the winning column
// the same way, so the XOR pairs words of the same rows.
//
// One launch per iteration, with the selection carried into the next launch
// so that no workgroup waits for another inside a launch.  Launch k:
//  1. reads the pair keys and the partial squared norms of r published by
//     launch k-1 (one of each per workgroup; the kernel boundary orders
//     them), sums the norms and runs the stop test for the k-1 steps taken
//     (||r||^2 <= eps^2 ||y||^2, or k-1 = T), then takes the largest key,
//     (idx, c*), as step k; every workgroup reaches the same result;
//  2. updates its columns' c_m with the Gram column of idx, stores them and
//     stores its best new key;
//  3. updates its own slice of rows of r in FP64 (r_n -/+ c*/sqrt(N)) and
//     stores the slice's partial ||r||^2;
//  4. in workgroup 0 only: x~_idx += c* (eq. 10), the trace entries and the
//     state (t, ||r||^2, stop reason).
// Keys and partial norms alternate between two halves by launch parity.  The
// first launch of a decode publishes the keys of c(0) and the norms of r = y;
// T steps take T+2 launches.  After the stop every launch returns at once.
#include <cstdlib>

#include "k_common.h"
#include "k_key2.h"
#include "mp_internal.h"

namespace mp {

constexpr int kSignThreads = 1024;
constexpr int kSignWaves = kSignThreads / kWave;
// Columns a wave handles at once: the same 128 bytes per lane in flight
// whatever the column length.
template <int CPL>
constexpr int kSignBatch = 8 / CPL;

// ---------------------------------------------------------------------------
// Set-up: the caller's packed bits (column m: ldw words) into the padded
// layout, bits of rows >= n cleared.
__global__ __launch_bounds__(256) void k_copy_signs(const uint32_t* __restrict__ in, int64_t ldw,
                                                    int n, int64_t m, int64_t ws,
                                                    uint32_t* __restrict__ out) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= m * ws) return;
  const int64_t col = i / ws;
  const int w = static_cast<int>(i % ws);
  const int row = 32 * w;
  uint32_t v = 0;
  if (row < n) {
    v = in[col * ldw + w];
    if (n - row < 32) v &= (1u << (n - row)) - 1u;
  }
  out[i] = v;
}

// Integer sum over the wave (exact; every lane receives it).
__device__ inline uint32_t wave_sum_u32(uint32_t v) {
  v += dpp_u32<kDppQuadSwap1>(v);
  v += dpp_u32<kDppQuadSwap2>(v);
  v += dpp_u32<kDppRowMirror>(v);
  v += dpp_u32<kDppRowHalfMirror>(v);
  v += static_cast<uint32_t>(__shfl_xor(static_cast<int>(v), 16, kWave));
  v += static_cast<uint32_t>(__shfl_xor(static_cast<int>(v), 32, kWave));
  return v;
}

// Rows of a 16-byte chunk whose signs differ between two columns.
__device__ inline uint32_t disagree(const v4u& a, const v4u& b) {
  return __builtin_popcount(a.x ^ b.x) + __builtin_popcount(a.y ^ b.y) +
         __builtin_popcount(a.z ^ b.z) + __builtin_popcount(a.w ^ b.w);
}

// ---------------------------------------------------------------------------
// c(0)_m = <y, psi_m> = (sum_n (1 - 2 b_nm) y_n) / sqrt(N) in FP64 for every
// column (eq. 9 at t = 0), and r = y in FP64.  One wave per column; lane l
// sums the rows of its chunks in increasing order, then the wave sums the
// lanes.  y is staged in LDS (32 ws floats, zero past n).
constexpr int kC0Threads = 256;
__global__ __launch_bounds__(kC0Threads) void k_sign_c0(const uint32_t* __restrict__ bits,
                                                        int64_t ws, int n, int64_t m,
                                                        const float* __restrict__ y,
                                                        double inv_sqrt_n, int64_t ld,
                                                        double* __restrict__ c64,
                                                        double* __restrict__ r64) {
  extern __shared__ float y_lds[];
  const int rows = static_cast<int>(32 * ws);
  for (int i = threadIdx.x; i < rows; i += kC0Threads) y_lds[i] = i < n ? y[i] : 0.0f;
  if (blockIdx.x == 0)
    for (int64_t i = threadIdx.x; i < ld; i += kC0Threads)
      r64[i] = i < n ? static_cast<double>(y[i]) : 0.0;
  __syncthreads();
  const int lane = threadIdx.x % kWave;
  const int nch = static_cast<int>(ws / 4);
  const int64_t stride = static_cast<int64_t>(gridDim.x) * (kC0Threads / kWave);
  for (int64_t col = static_cast<int64_t>(blockIdx.x) * (kC0Threads / kWave) +
                     threadIdx.x / kWave;
       col < m; col += stride) {
    const v4u* p = reinterpret_cast<const v4u*>(bits + col * ws);
    double acc = 0.0;
    for (int ch = lane; ch < nch; ch += kWave) {
      const v4u w = p[ch];
      const uint32_t word[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row0 = 128 * ch + 32 * q;
#pragma unroll 8
        for (int b = 0; b < 32; ++b) {
          const double v = static_cast<double>(y_lds[row0 + b]);
          acc += ((word[q] >> b) & 1u) ? -v : v;
        }
      }
    }
    acc = wave_sum(acc);
    if (lane == 0) c64[col] = acc * inv_sqrt_n;
  }
}

// ---------------------------------------------------------------------------
template <int CPL>
__global__ __launch_bounds__(kSignThreads) void k_mp_step_sign(
    const uint32_t* __restrict__ bits, int64_t ws, int n, int64_t m, int64_t ld,
    double* __restrict__ c64, double* __restrict__ r64, float* __restrict__ r32,
    double* __restrict__ rrp, double inv_n, double inv_sqrt_n, int cols_per_wg, int rows_per_wg,
    uint64_t* __restrict__ keys, long long k, long long max_iters, double thr,
    float* __restrict__ x, DevState* __restrict__ st, mp_trace tr) {
  __shared__ Key2 kred[kSignWaves];
  __shared__ double dred[kSignWaves];
  __shared__ int s_done;
  constexpr int B = kSignBatch<CPL>;
  const int lane = threadIdx.x % kWave;
  // the wave index as a wave-uniform value, so that per-column values sit in
  // scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) / kWave);
  const int64_t col0 = static_cast<int64_t>(blockIdx.x) * cols_per_wg;
  const int64_t col1 = col0 + cols_per_wg < m ? col0 + cols_per_wg : m;
  const int64_t row0 = static_cast<int64_t>(blockIdx.x) * rows_per_wg;  // this workgroup's rows
  const int64_t row1 = row0 + rows_per_wg < ld ? row0 + rows_per_wg : ld;
  const int nch = static_cast<int>(ws / 4);  // 16-byte chunks per column
  const int nk = static_cast<int>(gridDim.x);
  const int par = static_cast<int>(k & 1);
  const bool first = k == 0;
  const uint64_t* k_in = keys + (par ? 2 * nk : 0);
  uint64_t* k_out = keys + (par ? 0 : 2 * nk);
  const double* rr_in = rrp + (par ? nk : 0);
  double* rr_out = rrp + (par ? 0 : nk);

  // Requests first, all unconditional (clamped indices into valid memory;
  // what lies outside is discarded afterwards), so none waits for another.
  // The small ones go first, ahead of the columns' bits that every
  // workgroup requests at once: the stop flag, the previous keys and partial
  // norms, this wave's c and (wave 0) this workgroup's rows of r, then the
  // bits.
  const int done_v = __hip_atomic_load(&st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const int ki = static_cast<int>(threadIdx.x) < nk ? static_cast<int>(threadIdx.x) : nk - 1;
  Key2 kp{k_in[2 * ki], k_in[2 * ki + 1]};
  double rrq = rr_in[ki];
  double cm[B];
  int64_t colu[B];
#pragma unroll
  for (int u = 0; u < B; ++u) {
    const int64_t col = col0 + wave + u * kSignWaves;
    colu[u] = col < col1 ? col : col1 - 1;
    cm[u] = c64[colu[u]];
  }
  // wave 0: r_{k-1} of this workgroup's first 64 rows, one per lane
  double rq0 = 0.0;
  if (wave == 0) {
    const int64_t i = row0 + lane < ld ? row0 + lane : ld - 1;
    rq0 = r64[i];
  }
  v4u wb[B][CPL];
#pragma unroll
  for (int u = 0; u < B; ++u) {
    const v4u* p = reinterpret_cast<const v4u*>(bits + colu[u] * ws);
#pragma unroll
    for (int cc = 0; cc < CPL; ++cc) {
      const int ch = lane + kWave * cc;
      wb[u][cc] = p[ch < nch ? ch : nch - 1];
    }
  }
  if (first || static_cast<int>(threadIdx.x) >= nk) {
    kp = Key2{0, 0};
    rrq = 0.0;
  }
#pragma unroll
  for (int u = 0; u < B; ++u)
#pragma unroll
    for (int cc = 0; cc < CPL; ++cc)
      if (lane + kWave * cc >= nch) wb[u][cc] = v4u{0u, 0u, 0u, 0u};
  // one value of the flag for the whole workgroup, even in the launch in
  // which workgroup 0 sets it
  if (threadIdx.x == 0) s_done = done_v;
  __syncthreads();
  if (s_done) return;

  int idx = -1;
  double cs = 0.0;
  uint32_t wrow0 = 0;
  if (!first) {
    // Step k-1's residual: the stop test of the loop (the same sum, and so
    // the same decision, in every workgroup), then step k's atom.
    const double rr = block_sum<kSignThreads>(rrq, dred);
    const long long t = k - 1;  // steps taken so far
    const Key2 win = block_max_key2<kSignThreads>(kp, kred);
    idx = key2_index(win);
    cs = key2_value(win);
    int stop = -1;
    if (t > 0 && !(rr > thr)) stop = MP_STOP_CONVERGED;
    else if (t >= max_iters) stop = MP_STOP_MAX_ITERS;
    else if (idx < 0 || idx >= m) stop = kStopInternal;
    else if (cs == 0.0) stop = MP_STOP_STALLED;  // no atom correlates with r
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      if (t > 0) {
        if (t - 1 < tr.cap && tr.rr) tr.rr[t - 1] = rr;
        st->rr = rr;
      }
      st->t = t;
      if (stop != -1) {
        st->reason = stop;
        st->done = 1;
      } else {
        x[idx] += static_cast<float>(cs);
        if (t < tr.cap) {
          if (tr.idx) tr.idx[t] = idx;
          if (tr.coef) tr.coef[t] = static_cast<float>(cs);
        }
      }
    }
    if (stop != -1) return;

    // the winning column, chunk by chunk as this lane holds the others (and
    // in wave 0 the word of its first row)
    const v4u* pw = reinterpret_cast<const v4u*>(bits + static_cast<int64_t>(idx) * ws);
    if (wave == 0) {
      const int64_t i = row0 + lane < ld ? row0 + lane : ld - 1;
      wrow0 = bits[static_cast<int64_t>(idx) * ws + (i >> 5)];
    }
    v4u wv[CPL];
#pragma unroll
    for (int cc = 0; cc < CPL; ++cc) {
      const int ch = lane + kWave * cc;
      wv[cc] = pw[ch < nch ? ch : nch - 1];
    }
#pragma unroll
    for (int cc = 0; cc < CPL; ++cc)
      if (lane + kWave * cc >= nch) wv[cc] = v4u{0u, 0u, 0u, 0u};

    // c_m -= c* (N - 2 p_m) / N with p_m = popcount(b_idx XOR b_m); two
    // columns' counts share one 32-bit sum (each is at most N < 2^16)
    const double a = cs * inv_n;
#pragma unroll
    for (int u = 0; u < B; u += 2) {
      uint32_t pa = 0, pb = 0;
#pragma unroll
      for (int cc = 0; cc < CPL; ++cc) {
        pa += disagree(wb[u][cc], wv[cc]);
        pb += disagree(wb[u + 1][cc], wv[cc]);
      }
      const uint32_t sum = wave_sum_u32(pa | (pb << 16));
      cm[u] = __builtin_fma(-a, static_cast<double>(n - 2 * static_cast<int>(sum & 0xFFFFu)),
                            cm[u]);
      cm[u + 1] = __builtin_fma(-a, static_cast<double>(n - 2 * static_cast<int>(sum >> 16)),
                                cm[u + 1]);
    }
    if (lane == 0) {
#pragma unroll
      for (int u = 0; u < B; ++u)
        if (col0 + wave + u * kSignWaves < col1) c64[colu[u]] = cm[u];
    }
  }

  // Wave 0: this workgroup's rows of r (r_k = r_{k-1} -/+ c* / sqrt(N), rows
  // with a set bit get +, FP64) and their partial ||r_k||^2 for the next
  // launch's stop test; the first launch publishes the partials of r = y.
  if (wave == 0) {
    const double step = cs * inv_sqrt_n;
    const uint32_t* pw = bits + static_cast<int64_t>(idx < 0 ? 0 : idx) * ws;
    // the residual trace entry of step k - 1, if the trace asks for one
    float* rt = !first && tr.r && k - 1 < tr.cap ? tr.r + (k - 1) * tr.ldr : nullptr;
    double s = 0.0;
    for (int64_t i = row0 + lane; i < row1; i += kWave) {
      const bool lead = i == row0 + lane;
      double v = lead ? rq0 : r64[i];
      if (!first && i < n) {
        const uint32_t w = lead ? wrow0 : pw[i >> 5];
        v = ((w >> (i & 31)) & 1u) ? v + step : v - step;
        r64[i] = v;
        r32[i] = static_cast<float>(v);
        if (rt) rt[i] = static_cast<float>(v);
      }
      s += v * v;
    }
    s = wave_sum(s);
    if (lane == 0) rr_out[blockIdx.x] = s;
  }

  // this workgroup's best key for the next launch (a column read twice past
  // the range's end gives the same key twice)
  Key2 best{0, 0};
#pragma unroll
  for (int u = 0; u < B; ++u)
    best = key2_max(best, make_key2(cm[u], static_cast<int>(colu[u])));
  best = block_max_key2<kSignThreads>(best, kred);
  if (threadIdx.x == 0) {
    k_out[2 * blockIdx.x] = best.hi;
    k_out[2 * blockIdx.x + 1] = best.lo;
  }
}

// ---------------------------------------------------------------------------
// Persistent form: the whole decode in one launch, one workgroup per compute
// unit.  Each workgroup copies its columns' bits into LDS once
// (128 KB for 128 columns of N = 8192: the 32 MiB dictionary stays on chip
// across the 256 CUs for the whole decode), keeps its columns' c in
// registers and its rows of r (at most 64 kSignPersistRows) in registers of
// wave 0, so a step reads no dictionary bytes from memory.
//
// Step j does what launch j of k_mp_step_sign does, with the same arithmetic
// in the same order (bit-identical results).  In place of the kernel
// boundary between steps, each workgroup publishes its best key and partial
// ||r||^2 as kSignSlotWords words of the step's half of `slots`, each word
// carrying the step's tag beside 32 bits of the record, and reads every
// workgroup's words of the step before it goes on.
//
// The words are written and read with relaxed device-scope atomics (single
// 64-bit accesses, coherent across the XCDs); a reader takes a record once
// all its words carry the awaited tag, so no ordering between the words and
// no cache write-back or invalidation is needed.  Steps alternate between
// the two halves: a workgroup overwrites its words of step j - 2 only after
// reading every record of step j - 1, each of which its owner published
// after reading every record of step j - 2, so every reader of the old
// contents is done with them.  The epoch, new for every decode, keeps a
// word left by an earlier decode from matching.
//
// Every wait ends: the host launches this form only where the occupancy query
// shows every workgroup resident at once (one per CU, grid <= CUs), so all
// of them run together on an otherwise idle device; every workgroup runs the
// same steps and stops at the same one (the decision is taken from the same
// gathered values); and a poll that exceeds `spin_limit` tries marks the run
// failed (the sticky DevState::fail word) and its workgroup writes back its
// rows of r and leaves, after which every other workgroup's next poll times
// out too.  So a launch whose workgroups are not all resident (another
// kernel holding CUs) ends with MP_EDEVICE rather than waiting for ever.
// The launch is an ordinary one: a cooperative launch would add nothing the
// occupancy check does not give, and profilers have crashed at process exit
// after one.
constexpr int kSignPersistRows = 4;            // rows of r per lane of wave 0
constexpr int kSignPersistLds = 150 * 1024;    // dynamic LDS for the bits, at most

template <int CPL>
__global__ __launch_bounds__(kSignThreads) void k_sign_persist(
    const uint32_t* __restrict__ bits, int64_t ws, int n, int64_t m, int64_t ld,
    const double* __restrict__ c64, double* __restrict__ r64, float* __restrict__ r32,
    double inv_n, double inv_sqrt_n, int cols_per_wg, int rows_per_wg,
    unsigned long long* slots, unsigned epoch, long long spin_limit, long long max_iters, double thr,
    float* __restrict__ x, DevState* __restrict__ st, mp_trace tr) {
  extern __shared__ v4u s_bits[];  // this workgroup's columns, nch chunks each
  __shared__ Key2 kred[kSignWaves];
  __shared__ double dred[kSignWaves];
  __shared__ v4u s_win[kWave * CPL];  // the winning column's chunks
  __shared__ int s_fail;
  constexpr int B = kSignBatch<CPL>;
  constexpr int RPL = kSignPersistRows;
  const int lane = threadIdx.x % kWave;
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) / kWave);
  const int grid = static_cast<int>(gridDim.x);
  const int64_t col0 = static_cast<int64_t>(blockIdx.x) * cols_per_wg;
  const int64_t col1 = col0 + cols_per_wg < m ? col0 + cols_per_wg : m;
  const int64_t row0 = static_cast<int64_t>(blockIdx.x) * rows_per_wg;
  const int64_t row1 = row0 + rows_per_wg < ld ? row0 + rows_per_wg : ld;
  const int nch = static_cast<int>(ws / 4);
  const unsigned ep = (epoch % kSignEpochMod) << 20;  // the tag's epoch field

  // the columns' bits (contiguous: columns col0 .. col1-1) into LDS
  {
    const v4u* src = reinterpret_cast<const v4u*>(bits + col0 * ws);
    const int total = static_cast<int>(col1 - col0) * nch;
    for (int i = static_cast<int>(threadIdx.x); i < total; i += kSignThreads) s_bits[i] = src[i];
  }
  double cm[B];
  int colu[B];  // column index, clamped into the share as in k_mp_step_sign
#pragma unroll
  for (int u = 0; u < B; ++u) {
    const int64_t col = col0 + wave + u * kSignWaves;
    colu[u] = static_cast<int>(col < col1 ? col : col1 - 1);
    cm[u] = c64[colu[u]];
  }
  double rq[RPL];  // wave 0: rows row0 + lane + 64 q
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    const int64_t i = row0 + lane + kWave * q;
    rq[q] = (wave == 0 && i < row1) ? r64[i] : 0.0;
  }
  if (threadIdx.x == 0) s_fail = 0;
  __syncthreads();

  int idx = -1;
  double cs = 0.0;
  int x_pending = -1;  // workgroup 0: x~_idx += c* of the step, applied after publishing
  float x_add = 0.0f;
  for (long long j = 0;; ++j) {
    if (j > 0) {
      // every workgroup's key and partial norm of step j - 1
      Key2 kp{0, 0};
      double rrq = 0.0;
      if (static_cast<int>(threadIdx.x) < grid) {
        const unsigned want = ep | (static_cast<unsigned>(j) & 0xFFFFFu);  // step j - 1
        unsigned long long* w0 = slots + ((j - 1) & 1) * grid + threadIdx.x;
        unsigned long long w[kSignSlotWords];
        long long spins = 0;
        // poll the record's last word (stored last) alone, then read the
        // others: every workgroup polls every record, so one word per try
        // keeps the polling traffic down
        constexpr int L = kSignSlotWords - 1;
        for (;;) {
          w[L] = __hip_atomic_load(w0 + L * 2 * grid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (static_cast<unsigned>(w[L] >> 32) == want) {
            bool all = true;
#pragma unroll
            for (int q = 0; q < L; ++q) {
              w[q] = __hip_atomic_load(w0 + q * 2 * grid, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
              all = all && static_cast<unsigned>(w[q] >> 32) == want;
            }
            if (all) break;
          }
          if (++spins > spin_limit) {
            s_fail = 1;
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
        kp.hi = (w[0] << 32) | (w[1] & 0xFFFFFFFFull);
        kp.lo = w[2] & 0xFFFFFFFFull;
        rrq = __builtin_bit_cast(double, (w[3] << 32) | (w[4] & 0xFFFFFFFFull));
      }
      __syncthreads();
      if (s_fail) {
        // The failure is sticky: workgroup 0 may still store a regular stop
        // reason after this, so the host reads the fail word first.
        if (threadIdx.x == 0) {
          (void)__hip_atomic_fetch_or(&st->fail, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(&st->done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        break;  // rows of r as of the last step applied, written back below
      }
      // the stop test for the j - 1 steps taken, then step j's atom
      const double rr = block_sum<kSignThreads>(rrq, dred);
      const long long t = j - 1;
      const Key2 win = block_max_key2<kSignThreads>(kp, kred);
      idx = key2_index(win);
      cs = key2_value(win);
      int stop = -1;
      if (t > 0 && !(rr > thr)) stop = MP_STOP_CONVERGED;
      else if (t >= max_iters) stop = MP_STOP_MAX_ITERS;
      else if (idx < 0 || idx >= m) stop = kStopInternal;
      else if (cs == 0.0) stop = MP_STOP_STALLED;
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (t > 0) {
          if (t - 1 < tr.cap && tr.rr) tr.rr[t - 1] = rr;
          st->rr = rr;
        }
        st->t = t;
        if (stop != -1) {
          st->reason = stop;
          st->done = 1;
        } else {
          x_pending = idx;
          x_add = static_cast<float>(cs);
          if (t < tr.cap) {
            if (tr.idx) tr.idx[t] = idx;
            if (tr.coef) tr.coef[t] = static_cast<float>(cs);
          }
        }
      }
      if (stop != -1) break;

      // the winning column's chunks, once per workgroup (chunks past the
      // column zero)
      if (static_cast<int>(threadIdx.x) < kWave * CPL) {
        const int ch = static_cast<int>(threadIdx.x);
        const v4u* pw = reinterpret_cast<const v4u*>(bits + static_cast<int64_t>(idx) * ws);
        const v4u w = pw[ch < nch ? ch : nch - 1];
        s_win[ch] = ch < nch ? w : v4u{0u, 0u, 0u, 0u};
      }
      __syncthreads();
      v4u wv[CPL];
#pragma unroll
      for (int cc = 0; cc < CPL; ++cc) wv[cc] = s_win[lane + kWave * cc];

      // c_m -= c* (N - 2 p_m) / N, p_m = popcount(b_idx XOR b_m)
      const double a = cs * inv_n;
#pragma unroll
      for (int u = 0; u < B; u += 2) {
        uint32_t pa = 0, pb = 0;
#pragma unroll
        for (int cc = 0; cc < CPL; ++cc) {
          const int ch = lane + kWave * cc;
          const v4u za{0u, 0u, 0u, 0u};
          const v4u ba = ch < nch ? s_bits[(colu[u] - col0) * nch + ch] : za;
          const v4u bb = ch < nch ? s_bits[(colu[u + 1] - col0) * nch + ch] : za;
          pa += disagree(ba, wv[cc]);
          pb += disagree(bb, wv[cc]);
        }
        const uint32_t sum = wave_sum_u32(pa | (pb << 16));
        cm[u] = __builtin_fma(-a, static_cast<double>(n - 2 * static_cast<int>(sum & 0xFFFFu)),
                              cm[u]);
        cm[u + 1] = __builtin_fma(
            -a, static_cast<double>(n - 2 * static_cast<int>(sum >> 16)), cm[u + 1]);
      }
    }

    // wave 0: this workgroup's rows of r (r_j = r_{j-1} -/+ c* / sqrt(N) in
    // FP64, rows with a set bit get +) and their partial ||r_j||^2
    double part = 0.0;
    if (wave == 0) {
      const double step = cs * inv_sqrt_n;
      const uint32_t* win_words = reinterpret_cast<const uint32_t*>(s_win);
      // the residual trace entry of step j - 1, if the trace asks for one
      float* rt = j > 0 && tr.r && j - 1 < tr.cap ? tr.r + (j - 1) * tr.ldr : nullptr;
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < RPL; ++q) {
        const int64_t i = row0 + lane + kWave * q;
        if (i < row1) {
          double v = rq[q];
          if (j > 0 && i < n) {
            const uint32_t w = win_words[i >> 5];
            v = ((w >> (i & 31)) & 1u) ? v + step : v - step;
            rq[q] = v;
            if (rt) rt[i] = static_cast<float>(v);
          }
          s += v * v;
        }
      }
      part = wave_sum(s);
    }

    // this workgroup's best key; publish step j
    Key2 best{0, 0};
#pragma unroll
    for (int u = 0; u < B; ++u) best = key2_max(best, make_key2(cm[u], colu[u]));
    best = block_max_key2<kSignThreads>(best, kred);
    if (threadIdx.x == 0) {
      const unsigned long long tag =
          static_cast<unsigned long long>(ep | (static_cast<unsigned>(j + 1) & 0xFFFFFu)) << 32;
      const unsigned long long pr = __builtin_bit_cast(unsigned long long, part);
      const unsigned long long rec[kSignSlotWords] = {best.hi >> 32, best.hi & 0xFFFFFFFFull,
                                                      best.lo & 0xFFFFFFFFull, pr >> 32,
                                                      pr & 0xFFFFFFFFull};
      unsigned long long* w0 = slots + (j & 1) * grid + blockIdx.x;
#pragma unroll
      for (int q = 0; q < kSignSlotWords; ++q)
        __hip_atomic_store(w0 + q * 2 * grid, tag | rec[q], __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      if (x_pending >= 0) {
        x[x_pending] += x_add;
        x_pending = -1;
      }
    }
  }

  // r after the last step taken, rows below N
  if (wave == 0) {
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int64_t i = row0 + lane + kWave * q;
      if (i < row1 && i < n) {
        r64[i] = rq[q];
        r32[i] = static_cast<float>(rq[q]);
      }
    }
  }
}

int sign_chunks_per_lane(int64_t n) { return n <= 8192 ? 1 : 2; }

// The FP32 form's column shares, capped at the columns one workgroup scores
// (kSignWaves x kSignBatch: 128 columns with one chunk per lane, 64 with
// two), with more workgroups when M needs them.
CorrGeom sign_geometry(int64_t n, int64_t m, int num_cus) {
  CorrGeom g = corr_f32_geometry(m, num_cus);
  const int cap = sign_chunks_per_lane(n) == 1 ? kSignWaves * kSignBatch<1>
                                               : kSignWaves * kSignBatch<2>;
  if (g.cols_per_wg > cap) {
    g.cols_per_wg = cap;
    g.grid = static_cast<int>((m + cap - 1) / cap);
  }
  return g;
}

hipError_t launch_copy_signs(const uint32_t* in, int64_t ldw, int64_t n, int64_t m, int64_t ws,
                             uint32_t* out, hipStream_t s) {
  const int64_t total = m * ws;
  k_copy_signs<<<dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256), 0, s>>>(
      in, ldw, static_cast<int>(n), m, ws, out);
  return hipGetLastError();
}

hipError_t launch_sign_c0(const uint32_t* bits, int64_t ws, int64_t n, int64_t m, const float* y,
                          int64_t ld, double* c64, double* r64, hipStream_t s) {
  const size_t lds = sizeof(float) * 32 * static_cast<size_t>(ws);  // <= 64 KB (n <= 16384)
  int64_t blocks = (m + kC0Threads / kWave - 1) / (kC0Threads / kWave);
  if (blocks > 4096) blocks = 4096;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_sign_c0),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 64 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  k_sign_c0<<<dim3(static_cast<unsigned>(blocks)), dim3(kC0Threads), lds, s>>>(
      bits, ws, static_cast<int>(n), m, y, 1.0 / sqrt(static_cast<double>(n)), ld, c64, r64);
  return hipGetLastError();
}

bool sign_persist_fits(int64_t n, int64_t m, int64_t ld, int64_t ws, const CorrGeom& g,
                       int num_cus) {
  (void)m;
  const int64_t rows = (ld + g.grid - 1) / g.grid;
  const int64_t lds = static_cast<int64_t>(g.cols_per_wg) * ws * 4;
  return g.grid <= num_cus && g.grid <= kSignThreads && rows <= kWave * kSignPersistRows &&
         lds <= kSignPersistLds && n >= 1;
}

// The persistent kernel's LDS limit, set once per variant (the bits of a
// share need more than the default 64 KB).
static hipError_t sign_persist_attr(int which, const void* fn) {
  static bool attr_set[2] = {false, false};
  if (attr_set[which]) return hipSuccess;
  const hipError_t e =
      hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, kSignPersistLds);
  if (e == hipSuccess) attr_set[which] = true;
  return e;
}

static const void* sign_persist_fn(int64_t n) {
  return sign_chunks_per_lane(n) == 1 ? reinterpret_cast<const void*>(k_sign_persist<1>)
                                      : reinterpret_cast<const void*>(k_sign_persist<2>);
}

bool sign_persist_resident(int64_t n, int64_t ws, const CorrGeom& g, int num_cus) {
  const void* fn = sign_persist_fn(n);
  if (sign_persist_attr(sign_chunks_per_lane(n) == 1 ? 0 : 1, fn) != hipSuccess) return false;
  int per_cu = 0;
  const size_t lds = static_cast<size_t>(g.cols_per_wg) * static_cast<size_t>(ws) * 4;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kSignThreads, lds) != hipSuccess)
    return false;
  return static_cast<int64_t>(per_cu) * num_cus >= g.grid;
}

hipError_t launch_sign_persist(const uint32_t* bits, int64_t ws, int64_t n, int64_t m, int64_t ld,
                               const double* c64, double* r64, float* r32, const CorrGeom& g,
                               unsigned long long* slots, unsigned epoch, long long max_iters,
                               double thr, float* x, DevState* st, mp_trace tr, hipStream_t s) {
  const double inv_n = 1.0 / static_cast<double>(n);
  const double inv_sqrt_n = 1.0 / sqrt(static_cast<double>(n));
  int rows_per_wg = static_cast<int>((ld + g.grid - 1) / g.grid);
  int cols_per_wg = g.cols_per_wg;
  int nn = static_cast<int>(n);
  // polls per wait before the run is marked failed; MP_SIGN_SPIN_LIMIT (a
  // positive integer) overrides it, so that tests can drive the failure path
  long long spin_limit = 1ll << 22;
  if (const char* env = getenv("MP_SIGN_SPIN_LIMIT")) {
    const long long v = atoll(env);
    if (v > 0) spin_limit = v;
  }
  const size_t lds = static_cast<size_t>(g.cols_per_wg) * static_cast<size_t>(ws) * 4;
  const int cap = sign_chunks_per_lane(n) == 1 ? kSignWaves * kSignBatch<1>
                                               : kSignWaves * kSignBatch<2>;
  if (g.cols_per_wg > cap || rows_per_wg > kWave * kSignPersistRows ||
      lds > static_cast<size_t>(kSignPersistLds) || g.grid > kSignThreads)
    return hipErrorInvalidValue;
  void* args[] = {&bits, &ws, &nn, &m, &ld, &c64, &r64, &r32, const_cast<double*>(&inv_n),
                  const_cast<double*>(&inv_sqrt_n), &cols_per_wg, &rows_per_wg, &slots, &epoch,
                  &spin_limit, &max_iters, &thr, &x, &st, &tr};
  const void* fn = sign_persist_fn(n);
  if (hipError_t e = sign_persist_attr(sign_chunks_per_lane(n) == 1 ? 0 : 1, fn); e != hipSuccess)
    return e;
  return hipLaunchKernel(fn, dim3(g.grid), dim3(kSignThreads), args, lds, s);
}

hipError_t launch_mp_step_sign(const uint32_t* bits, int64_t ws, int64_t n, int64_t m, int64_t ld,
                               double* c64, double* r64, float* r32, double* rrp,
                               const CorrGeom& g, uint64_t* keys, long long k, long long max_iters,
                               double thr, float* x, DevState* st, mp_trace tr, hipStream_t s) {
  const double inv_n = 1.0 / static_cast<double>(n);
  const double inv_sqrt_n = 1.0 / sqrt(static_cast<double>(n));
  const int rows_per_wg = static_cast<int>((ld + g.grid - 1) / g.grid);
  // a workgroup scores kSignWaves x kSignBatch columns: a larger share
  // would leave columns unscored
  const int cap = sign_chunks_per_lane(n) == 1 ? kSignWaves * kSignBatch<1>
                                               : kSignWaves * kSignBatch<2>;
  if (g.cols_per_wg > cap || g.grid > kSignThreads) return hipErrorInvalidValue;
  if (sign_chunks_per_lane(n) == 1)
    k_mp_step_sign<1><<<dim3(g.grid), dim3(kSignThreads), 0, s>>>(
        bits, ws, static_cast<int>(n), m, ld, c64, r64, r32, rrp, inv_n, inv_sqrt_n,
        g.cols_per_wg, rows_per_wg, keys, k, max_iters, thr, x, st, tr);
  else
    k_mp_step_sign<2><<<dim3(g.grid), dim3(kSignThreads), 0, s>>>(
        bits, ws, static_cast<int>(n), m, ld, c64, r64, r32, rrp, inv_n, inv_sqrt_n,
        g.cols_per_wg, rows_per_wg, keys, k, max_iters, thr, x, st, tr);
  return hipGetLastError();
}

}  // namespace mp
