// Matching Pursuit on the Bernoulli dictionary of eq. 13 held as one sign bit
// per entry, for gfx950.
//
// psi_nm = (1 - 2 b_nm) / sqrt(N).  With the signs s_nm = 1 - 2 b_nm the
// correlation of eq. 9 is c_m = (sum_n s_nm r_n) / sqrt(N): no products, and
// a column is N bits instead of 4N bytes, so the pass reads 32x less than the
// FP32 one and is bound by the arithmetic instead of HBM.
//
// Signed sums by table look-up.  Rows are taken in groups of four; for every
// group g each workgroup tabulates in LDS the 16 signed sums
//   T_g[b] = sum_{k<4} (bit k of b set ? -r_{4g+k} : +r_{4g+k}),
// after which a column's signed sum is one LDS read and one add per four rows:
//   sum_n s_nm r_n = sum_g T_g[nibble g of column m].
//
// Layout of the sign bits (built once by k_tile_signs from the packed input):
// the wave that handles a column reads all of it with one load of J words
// per lane (J = 1, 2 or 4; N <= 2048 J).  Nibble k of lane l's word j holds
// the four bits of group g = l + 64 (8 j + k), bit i of the nibble being row
// 4 g + i.  The table is stored plane by plane, T_g[b] at b G + g with
// G = 512 J: every group a lane looks up is congruent to the lane mod 64 and
// G is a multiple of 64, so the 64 reads of a look-up fall in 64 different
// LDS banks whatever the nibbles are.
//
// One MP iteration is one launch; the selection of a pass is made at the
// start of the next launch, by every workgroup alike (see k_mp_step_sign).
#include "k_common.h"
#include "mp_internal.h"

namespace mp {

constexpr int kSignThreads = 1024;
constexpr int kSignWaves = kSignThreads / kWave;
constexpr int kSignBatch = 8;  // columns a wave loads before it sums them

typedef unsigned v2u __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------------------
// Set-up: packed input (column m: ldw words, bit q of word w = row 32 w + q)
// -> lane-interleaved tiles (column m: 64 J words, lane l's J words together).
// Bits of rows >= n are cleared.
__global__ __launch_bounds__(256) void k_tile_signs(const uint32_t* __restrict__ in, int64_t ldw,
                                                    int n, int64_t m, int J,
                                                    uint32_t* __restrict__ out) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  const int64_t per_col = 64 * J;
  if (i >= m * per_col) return;
  const int64_t col = i / per_col;
  const int rem = static_cast<int>(i % per_col);
  const int l = rem / J, j = rem % J;
  const uint32_t* src = in + col * ldw;
  uint32_t w = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int row = 4 * (l + 64 * (8 * j + k));
    if (row >= n) continue;
    uint32_t nib = (src[row >> 5] >> (row & 31)) & 0xFu;  // a group never straddles a word
    if (n - row < 4) nib &= (1u << (n - row)) - 1u;
    w |= nib << (4 * k);
  }
  out[i] = w;
}

// The reverse, for mp_get_storage: tiles -> packed (ceil(n/32) words per column).
__global__ __launch_bounds__(256) void k_untile_signs(const uint32_t* __restrict__ tiles, int n,
                                                      int64_t m, int J,
                                                      uint32_t* __restrict__ out) {
  const int64_t words = (n + 31) / 32;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= m * words) return;
  const int64_t col = i / words;
  const int w = static_cast<int>(i % words);
  const uint32_t* src = tiles + col * 64 * J;
  uint32_t v = 0;
#pragma unroll
  for (int q = 0; q < 32; q += 4) {
    const int row = 32 * w + q;
    if (row >= n) break;
    const int g = row >> 2, t = g >> 6;
    v |= ((src[(g & 63) * J + (t >> 3)] >> (4 * (t & 7))) & 0xFu) << q;
  }
  out[i] = v;
}

// ---------------------------------------------------------------------------
template <int J>
__device__ inline void load_sign_words(const uint32_t* __restrict__ p, uint32_t (&w)[J]) {
  if constexpr (J == 4) {
    const v4u v = *reinterpret_cast<const v4u*>(p);
    w[0] = v.x;
    w[1] = v.y;
    w[2] = v.z;
    w[3] = v.w;
  } else if constexpr (J == 2) {
    const v2u v = *reinterpret_cast<const v2u*>(p);
    w[0] = v.x;
    w[1] = v.y;
  } else {
    w[0] = *p;
  }
}

// One launch per MP iteration, with the selection carried into the next
// launch so that no workgroup hands off to another inside a launch.  Launch k
// finishes iteration k-1 and runs the correlation pass of iteration k:
//  1. every workgroup reads the keys of pass k-1 (one per workgroup, stored
//     by launch k-1; the kernel boundary orders them) and r_{k-1}; all take
//     the same winner, the largest key, and compute the same
//     r_k = r_{k-1} - c psi_idx (eq. 11: r_n -/+ c / sqrt(N)) for every row;
//  2. workgroup 0 alone stores r_k for launch k+1, adds c to x~_idx
//     (eq. 10), writes the trace entry, counts t (eq. 12) and runs the stop
//     test on ||r_k||^2 in FP64, with every value it reads requested
//     together with the launch's first loads or the winner's bits;
//  3. every workgroup builds the table from r_k, runs the pass over its
//     columns and stores its best key for launch k+1.
// r and the keys alternate between two halves by launch parity.  The first
// launch of a decode has no pass to finish (`first`).  After the stop every
// launch returns at once; in the launch that sets it, the other workgroups
// may still run a pass whose keys are never read.
//
// Workgroup b takes columns [b cols_per_wg, (b+1) cols_per_wg); wave w of it
// the columns w, w+16, ... of that range, kSignBatch at a time (past the
// range's end the last column is read again, which leaves the maximum
// unchanged).  `width` is always 4, the nibble width: taken as an argument it
// keeps each nibble read a single bit-field extract, which the address add
// can then absorb (with a constant width the compiler splits it into a shift
// and a mask).
template <int J>
__global__ __launch_bounds__(kSignThreads) void k_mp_step_sign(
    const uint32_t* __restrict__ tiles, int n, int64_t m, int64_t ld, float* __restrict__ rbuf,
    float inv_sqrt_n, int cols_per_wg, unsigned width, uint64_t* __restrict__ keys, int parity,
    int first, float* __restrict__ x, DevState* __restrict__ st, mp_trace tr) {
  constexpr int G = 512 * J;  // groups of four rows covered by one column load
  constexpr int GPT = (G + kSignThreads - 1) / kSignThreads;  // groups per thread
  extern __shared__ float lut[];  // 16 planes of G floats
  __shared__ uint64_t kred[kSignWaves];
  __shared__ double dred[kSignWaves];
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int64_t col0 = static_cast<int64_t>(blockIdx.x) * cols_per_wg;
  const int64_t col1 = col0 + cols_per_wg < m ? col0 + cols_per_wg : m;
  const int64_t step = kSignWaves * kSignBatch;
  const int ld4 = static_cast<int>(ld / 4);  // r: ld floats, rows >= n zero
  const v4f* r_in = reinterpret_cast<const v4f*>(rbuf + (parity ? ld : 0));
  v4f* r_out = reinterpret_cast<v4f*>(rbuf + (parity ? 0 : ld));
  const uint64_t* k_in = keys + (parity ? gridDim.x : 0);
  uint64_t* k_out = keys + (parity ? 0 : gridDim.x);

  // Requests first, all of them unconditional (clamped indices into valid
  // memory; what lies outside is zeroed afterwards), so none waits for
  // another: the stop flag, r_{k-1} for this thread's groups (g = i + 1024 t,
  // rows 4g..4g+3), the previous pass's keys and the first batch of columns.
  // The flag is broadcast from thread 0, so the whole workgroup sees one
  // value even in the launch in which workgroup 0 sets it.
  __shared__ int s_done;
  const int done_v = __hip_atomic_load(&st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // workgroup 0 keeps the run's state: what its bookkeeping reads, now
  long long st_t = 0, st_max = 0;
  double st_thr = 0.0;
  if (blockIdx.x == 0) {
    st_t = st->t;
    st_max = st->max_iters;
    st_thr = st->thr;
  }
  v4f q[GPT];
#pragma unroll
  for (int t = 0; t < GPT; ++t) {
    const int g = threadIdx.x + t * kSignThreads;
    q[t] = r_in[g < ld4 ? g : ld4 - 1];
  }
  const int nkeys = static_cast<int>(gridDim.x);  // <= kSignThreads
  uint64_t kprev = k_in[static_cast<int>(threadIdx.x) < nkeys ? threadIdx.x : nkeys - 1];
  uint32_t w[kSignBatch][J];
  int64_t cb = col0 + wave;
#pragma unroll
  for (int u = 0; u < kSignBatch; ++u) {
    int64_t col = cb + u * kSignWaves;
    col = col < col1 ? col : col1 - 1;
    load_sign_words<J>(tiles + col * 64 * J + lane * J, w[u]);
  }
#pragma unroll
  for (int t = 0; t < GPT; ++t)
    if (threadIdx.x + t * kSignThreads >= ld4) q[t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
  if (first || static_cast<int>(threadIdx.x) >= nkeys) kprev = 0;
  if (threadIdx.x == 0) s_done = done_v;
  __syncthreads();
  if (s_done) return;
  if (!first) {
    // finish iteration k-1: the winner, then r_k in registers
    const uint64_t win = block_max<kSignThreads>(kprev, kred);
    const int idx = key_index(win);
    const float c = key_value(win);
    if (idx < 0 || idx >= m || c == 0.0f) {  // c = 0: no atom correlates with r
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->done = 1;
        st->reason = (idx < 0 || idx >= m) ? kStopInternal : MP_STOP_STALLED;
      }
      return;
    }
    const float a = c * inv_sqrt_n;
    const uint32_t* wc = tiles + static_cast<int64_t>(idx) * 64 * J;
    const float x_old = blockIdx.x == 0 ? x[idx] : 0.0f;  // requested with the winner's bits
    uint32_t word[GPT];
#pragma unroll
    for (int t = 0; t < GPT; ++t) {
      int g = threadIdx.x + t * kSignThreads;
      g = g < ld4 ? g : ld4 - 1;  // rows past ld are not updated below
      word[t] = wc[(g & 63) * J + ((g >> 6) >> 3)];
    }
    double s = 0.0;
#pragma unroll
    for (int t = 0; t < GPT; ++t) {
      const int g = threadIdx.x + t * kSignThreads;
      if (g < ld4) {
        const uint32_t nib = word[t] >> (4 * ((g >> 6) & 7));
        const int row = 4 * g;
        v4f o;
        o.x = row + 0 < n ? ((nib & 1u) ? q[t].x + a : q[t].x - a) : 0.0f;
        o.y = row + 1 < n ? ((nib & 2u) ? q[t].y + a : q[t].y - a) : 0.0f;
        o.z = row + 2 < n ? ((nib & 4u) ? q[t].z + a : q[t].z - a) : 0.0f;
        o.w = row + 3 < n ? ((nib & 8u) ? q[t].w + a : q[t].w - a) : 0.0f;
        q[t] = o;
        s += static_cast<double>(o.x) * o.x + static_cast<double>(o.y) * o.y +
             (static_cast<double>(o.z) * o.z + static_cast<double>(o.w) * o.w);
      }
    }
    if (blockIdx.x == 0) {
      // r_k for the next launch, x~_idx += c (eq. 10), the trace entry,
      // t + 1 (eq. 12) and the stop test on the FP64 ||r_k||^2
#pragma unroll
      for (int t = 0; t < GPT; ++t) {
        const int g = threadIdx.x + t * kSignThreads;
        if (g < ld4) r_out[g] = q[t];
      }
      const double rr = block_sum<kSignThreads>(s, dred);
      if (threadIdx.x == 0) {
        x[idx] = x_old + c;
        if (st_t < tr.cap) {
          if (tr.idx) tr.idx[st_t] = idx;
          if (tr.coef) tr.coef[st_t] = c;
          if (tr.rr) tr.rr[st_t] = rr;
        }
        st->t = st_t + 1;
        st->rr = rr;
        st->r_sel = parity ^ 1;
        if (!(rr > st_thr)) {
          st->reason = MP_STOP_CONVERGED;
          st->done = 1;
        } else if (st_t + 1 >= st_max) {
          st->reason = MP_STOP_MAX_ITERS;
          st->done = 1;
        }
      }
    }
  } else if (blockIdx.x == 0) {
#pragma unroll
    for (int t = 0; t < GPT; ++t) {
      const int g = threadIdx.x + t * kSignThreads;
      if (g < ld4) r_out[g] = q[t];
    }
    if (threadIdx.x == 0) st->r_sel = parity ^ 1;
  }

  // T_g[b] from r_k: bits 0 and 1 of b sign rows 4g and 4g+1 (pa), bits 2
  // and 3 rows 4g+2 and 4g+3 (pb)
#pragma unroll
  for (int t = 0; t < GPT; ++t) {
    const int g = threadIdx.x + t * kSignThreads;
    if (g < G) {
      const v4f v = q[t];
      const float pa[4] = {v.x + v.y, v.y - v.x, v.x - v.y, -(v.x + v.y)};
      const float pb[4] = {v.z + v.w, v.w - v.z, v.z - v.w, -(v.z + v.w)};
#pragma unroll
      for (int b = 0; b < 16; ++b) lut[b * G + g] = pa[b & 3] + pb[b >> 2];
    }
  }
  __syncthreads();

  // look-up address of nibble value v for this lane: v * 4G bytes (the plane)
  // + 4 * lane (its bank); the group's offset 256 (8j + k) is a constant
  const uint32_t lane4 = 4u * static_cast<uint32_t>(lane);
  const char* lut_b = reinterpret_cast<const char*>(lut);
  uint64_t best = 0;
  while (cb < col1) {
    float acc[kSignBatch];
#pragma unroll
    for (int j = 0; j < J; ++j) {
#pragma unroll
      for (int k = 0; k < 8; ++k) {
#pragma unroll
        for (int u = 0; u < kSignBatch; ++u) {
          const uint32_t nib = __builtin_amdgcn_ubfe(w[u][j], 4 * k, width);
          const uint32_t off = nib * (4u * G) + lane4;
          const float v = *reinterpret_cast<const float*>(lut_b + off + 256 * (8 * j + k));
          acc[u] = (j == 0 && k == 0) ? v : acc[u] + v;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kSignBatch; ++u) {
      int64_t col = cb + u * kSignWaves;
      col = col < col1 ? col : col1 - 1;
      const uint64_t key = make_key(wave_sum(acc[u]) * inv_sqrt_n, static_cast<int>(col));
      best = key > best ? key : best;
    }
    cb += step;
    if (cb < col1) {
#pragma unroll
      for (int u = 0; u < kSignBatch; ++u) {
        int64_t col = cb + u * kSignWaves;
        col = col < col1 ? col : col1 - 1;
        load_sign_words<J>(tiles + col * 64 * J + lane * J, w[u]);
      }
    }
  }
  best = block_max<kSignThreads>(best, kred);
  if (threadIdx.x == 0) k_out[blockIdx.x] = best;
}

int sign_words_per_lane(int64_t n) { return n <= 2048 ? 1 : (n <= 4096 ? 2 : 4); }

hipError_t launch_tile_signs(const uint32_t* in, int64_t ldw, int64_t n, int64_t m, int J,
                             uint32_t* out, hipStream_t s) {
  const int64_t total = m * 64 * J;
  k_tile_signs<<<dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256), 0, s>>>(
      in, ldw, static_cast<int>(n), m, J, out);
  return hipGetLastError();
}

hipError_t launch_untile_signs(const uint32_t* tiles, int64_t n, int64_t m, int J, uint32_t* out,
                               hipStream_t s) {
  const int64_t total = m * ((n + 31) / 32);
  k_untile_signs<<<dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256), 0, s>>>(
      tiles, static_cast<int>(n), m, J, out);
  return hipGetLastError();
}

template <int J>
static hipError_t launch_step_sign_j(const uint32_t* tiles, int64_t n, int64_t m, int64_t ld,
                                     float* rbuf, float inv_sqrt_n, const CorrGeom& g,
                                     uint64_t* keys, int parity, int first, float* x,
                                     DevState* st, mp_trace tr, hipStream_t s) {
  const size_t lds = sizeof(float) * 16 * 512 * J;
  static bool attr_set = false;  // tables above 64 KB need the opt-in limit
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_mp_step_sign<J>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(lds));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  k_mp_step_sign<J><<<dim3(g.grid), dim3(kSignThreads), lds, s>>>(
      tiles, static_cast<int>(n), m, ld, rbuf, inv_sqrt_n, g.cols_per_wg, 4u, keys, parity,
      first, x, st, tr);
  return hipGetLastError();
}

hipError_t launch_mp_step_sign(const uint32_t* tiles, int J, int64_t n, int64_t m, int64_t ld,
                               float* rbuf, float inv_sqrt_n, const CorrGeom& g, uint64_t* keys,
                               int parity, int first, float* x, DevState* st, mp_trace tr,
                               hipStream_t s) {
  switch (J) {
    case 1:
      return launch_step_sign_j<1>(tiles, n, m, ld, rbuf, inv_sqrt_n, g, keys, parity, first, x,
                                   st, tr, s);
    case 2:
      return launch_step_sign_j<2>(tiles, n, m, ld, rbuf, inv_sqrt_n, g, keys, parity, first, x,
                                   st, tr, s);
    case 4:
      return launch_step_sign_j<4>(tiles, n, m, ld, rbuf, inv_sqrt_n, g, keys, parity, first, x,
                                   st, tr, s);
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace mp
