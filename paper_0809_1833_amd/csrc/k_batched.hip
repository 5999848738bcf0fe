// Batched Matching Pursuit: many signals against one shared dictionary.
//
// Layouts read by the product: the dictionary's BF16 copy in tiles of 16
// atoms x 32 K elements, each tile 1 KB contiguous (atom block, then K
// chunk, then the 16 atoms' 32 elements), so one MFMA operand load reads
// 1 KB in one piece; the residuals' BF16 copy with leading dimension ldq =
// ld + 32 elements, which spreads the 16 signal rows of one operand load
// over the memory channels (a stride of exactly 4 KB sends them all to one).
//
// One round performs one MP iteration (Section 3, eqs. 9-12) for every
// signal still active.  The correlations of all active signals with all
// atoms are one matrix product C = Psi^T R (the residuals as columns), run
// on the BF16 matrix cores with FP32 accumulation; its epilogue keeps, for
// every signal, the 8 best atoms of each 64-atom tile.  A second kernel, one
// workgroup per active signal, merges those into the signal's 8 best
// candidates, re-scores them against the FP32 columns and the FP32 residual,
// takes the best (smallest index on ties, eq. 16) and updates x~, r and the
// FP64 stopping test for that signal, and stores whether the signal goes on.
// Signals stop at their own iteration.  The list of active signals is
// compacted one round behind: an extra workgroup of round r's select drops
// the signals that stopped in round r-1 (their flags, written before the
// kernel boundary), so round r+1 covers at most the signals that stop in
// round r, which its select skips.  No workgroup waits for another and no
// atomics are used.
#include <type_traits>

#include "k_common.h"
#include "k_lowp.h"
#include "mp_internal.h"

namespace mp {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 v8bf;

constexpr int kBThreads = 256;              // 4 waves (init and compaction)
constexpr int kBSelThreads = 512;           // 8 waves: one per re-scored candidate
constexpr int kBSelWaves = kBSelThreads / kWave;
constexpr int kBTopK = kTopK;

// ---------------------------------------------------------------------------
// Init: every signal slot b < B.  r = y (zero padded), its BF16 copy, x~ = 0,
// ||y||^2 in FP64, the loop's pre-test.  One workgroup per slot.
__global__ __launch_bounds__(kBThreads) void k_binit(
    const float* __restrict__ Y, int64_t ldy, int64_t n, int64_t ld, float* __restrict__ X,
    int64_t ldx, int64_t m, float* __restrict__ R32, uint16_t* __restrict__ Rq, int64_t ldq,
    BSlot* __restrict__ slots, const long long* __restrict__ tcap, long long tcap_all,
    double eps) {
  __shared__ double red[kBThreads / kWave];
  const int64_t b = blockIdx.x;
  const float* y = Y + b * ldy;
  float* r = R32 + b * ld;
  uint16_t* rq = Rq + b * ldq;
  float* x = X + b * ldx;
  for (int64_t j = threadIdx.x; j < m; j += kBThreads) x[j] = 0.0f;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < ld; i += kBThreads) {
    const float v = i < n ? y[i] : 0.0f;
    r[i] = v;
    rq[i] = bf16_rne(v);
    s += static_cast<double>(v) * v;
  }
  const double yy = block_sum<kBThreads>(s, red);
  if (threadIdx.x == 0) {
    BSlot d{};
    d.yy = yy;
    d.rr = yy;
    d.thr = eps * eps * yy;
    d.t = 0;
    d.max_iters = tcap ? tcap[b] : tcap_all;
    d.reason = MP_STOP_CONVERGED;
    d.done = 0;
    if (!__builtin_isfinite(yy)) {
      d.done = 1;
      d.reason = kStopNonFinite;
    } else if (yy == 0.0) {
      d.done = 1;
      d.reason = MP_STOP_ZERO_INPUT;
    } else if (!(yy > d.thr)) {
      d.done = 1;
      d.reason = MP_STOP_CONVERGED;
    } else if (d.max_iters <= 0) {
      d.done = 1;
      d.reason = MP_STOP_MAX_ITERS;
    }
    slots[b] = d;
  }
}

// The BF16 dictionary in product tiles: element (atom a, row k) goes to
// tile (a / 16, k / 32), position (a % 16) * 32 + k % 32; atoms past m (up to
// the next multiple of 16) are zero.  One 256-thread workgroup per tile row
// block of 16 atoms, looping over the K chunks.
__global__ __launch_bounds__(256) void k_tile_bf16(const float* __restrict__ psi, int64_t ld,
                                                   int64_t m, uint16_t* __restrict__ out) {
  const int64_t blk = blockIdx.x;
  const int64_t nchunks = ld / 32;
  for (int64_t e = threadIdx.x; e < nchunks * 512; e += 256) {
    const int64_t chunk = e / 512, within = e % 512;
    const int64_t a = blk * 16 + within / 32, k = chunk * 32 + within % 32;
    out[blk * 16 * ld + e] = a < m ? bf16_rne(psi[a * ld + k]) : uint16_t{0};
  }
}

// Stable compaction (one workgroup of NT threads): the positions j < n_in
// with keep(j) go, in order, to list_out (their slot list_in[j], or j itself
// when list_in is null) and src_out (j, when not null); returns the count in
// every thread.
template <int NT, typename Keep>
__device__ int compact_list(const int* __restrict__ list_in, int n_in, Keep keep,
                            int* __restrict__ list_out, int* __restrict__ src_out) {
  __shared__ int wsum[NT / kWave];
  __shared__ int base_s;
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  if (threadIdx.x == 0) base_s = 0;
  __syncthreads();
  for (int j0 = 0; j0 < n_in; j0 += NT) {
    const int j = j0 + threadIdx.x;
    const int jc = j < n_in ? j : 0;  // both loads issued together, in bounds
    const int slot = list_in ? list_in[jc] : j;
    const bool k = j < n_in && keep(jc);
    const unsigned long long bal = __ballot(k);
    const int before = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wave] = __popcll(bal);
    __syncthreads();
    int off = base_s;
    for (int w = 0; w < wave; ++w) off += wsum[w];
    if (k) {
      list_out[off + before] = slot;
      if (src_out) src_out[off + before] = j;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int tot = 0;
      for (int w = 0; w < NT / kWave; ++w) tot += wsum[w];
      base_s += tot;
    }
    __syncthreads();
  }
  return base_s;
}

// After init: the running slots into list 0 (round 0's), their source
// positions the identity and the flags "running before round 0" set.
// keep holds four arrays of cap ints: flags of rounds with parity 0 and 1,
// then source positions of lists 0 and 1.
__global__ __launch_bounds__(kBThreads) void k_bcompact_init(int nslots, const BSlot* slots,
                                                             int* act, int* keep, int64_t cap,
                                                             BState* bs) {
  const int n = compact_list<kBThreads>(nullptr, nslots,
                                        [&](int j) { return slots[j].done == 0; }, act, nullptr);
  for (int j = threadIdx.x; j < n; j += kBThreads) {
    keep[cap + j] = 1;      // flags of "round -1"
    keep[2 * cap + j] = j;  // list 0's source positions
  }
  if (threadIdx.x == 0) bs->n_active[0] = n;
}

// ---------------------------------------------------------------------------
// Product tile: (16 TI) atoms x 64 signals per workgroup of 4 waves; TI = 4
// when many signals are active, TI = 2 (twice the workgroups) when few are.
// Every wave computes the whole tile as TI x 4 MFMA 16x16 blocks (K = 32 per
// MFMA) over its share of K: wave w takes the K-steps w, w + 4, w + 8, ...
// (neighbouring waves read neighbouring bytes of the same cache lines).
// Operands come straight from global memory (the BF16 dictionary stays in
// the last-level cache across rounds, the residuals in L2): lane l loads 16
// contiguous bytes of atom row (l % 16) and of signal column (l % 16) at K
// offset 8 * (l / 16).  Rows past the last atom and columns past the last
// active signal load the last valid row or column instead: an operand row
// only reaches its own row (column) of the product, which the epilogue
// skips, so no load needs a predicate and the loads of the next kBPre
// K-steps stay in flight in a register ring while the current step's MFMAs
// run (scheduling barriers keep each step's loads behind its MFMAs, so the
// oldest slot is the only one waited for; two waves per SIMD fit).  The four partial tiles are summed in LDS in a fixed order,
// ((w0 + w2) + (w1 + w3)); then thread (wave, lane) sorts the keys of rows
// [wave * TM/4, (wave + 1) * TM/4) of signal column `lane` with sorting
// networks, and the four sorted lists are merged pairwise into the signal's
// 8 best atoms of the tile (descending), written to `partials`.
constexpr int kBCorrThreads = 256;
constexpr int kBCorrWaves = kBCorrThreads / kWave;   // K split
constexpr int kBCorrTileB = 64;                      // signals per workgroup
constexpr int kBPre = 4;                             // K-steps in flight per wave

// Each signal's 8 best atoms of a product tile (the epilogue of the product
// kernels): `ct` holds the tile's TM x 64 correlations; thread (wave, lane)
// of waves 0-3 sorts the keys of rows [wave * TM/4, (wave + 1) * TM/4) of
// signal column `lane` with sorting networks, and the four sorted lists are
// merged pairwise into the signal's 8 best atoms (descending), written to
// `partials`.  Every thread of the workgroup calls it (barriers).
template <int TM>
__device__ void tile_top8(const float (*ct)[kBCorrTileB + 1],
                          uint64_t (&lists)[2][kBTopK][kBCorrTileB], int64_t m0, int64_t m,
                          int nact, int j0, int lane, int wave, uint64_t* __restrict__ partials,
                          int mtiles) {
  constexpr int RP = TM / 4;  // rows per thread of waves 0-3: 32, 16, 8 or 4
  static_assert(RP == 32 || RP == 16 || RP == 8 || RP == 4, "tile height");
  uint64_t L[kBTopK];
  if (wave < 4) {
    // groups of 8 rows (4 rows and 4 empty keys in a 16-atom tile), each
    // sorted, merged into the running top 8
#pragma unroll
    for (int g = 0; g < (RP + kBTopK - 1) / kBTopK; ++g) {
      uint64_t h[kBTopK];
#pragma unroll
      for (int q = 0; q < kBTopK; ++q) {
        const int rl = g * kBTopK + q;  // row of this thread's share
        const int rr = wave * RP + (rl < RP ? rl : 0);
        const int64_t atom = m0 + rr;
        h[q] = rl < RP && atom < m ? make_key(ct[rr][lane], static_cast<int>(atom)) : 0ull;
      }
      sort8_keys(h);
      if (g == 0) {
#pragma unroll
        for (int q = 0; q < kBTopK; ++q) L[q] = h[q];
      } else {
        merge8_keys(L, h);
      }
    }
  }
  // waves 2, 3 hand their lists to waves 0, 1; then wave 1 to wave 0 (waves
  // past 3, if any, only take part in the barriers)
  if (wave >= 2 && wave < 4)
#pragma unroll
    for (int q = 0; q < kBTopK; ++q) lists[wave - 2][q][lane] = L[q];
  __syncthreads();
  if (wave < 2) {
    uint64_t o[kBTopK];
#pragma unroll
    for (int q = 0; q < kBTopK; ++q) o[q] = lists[wave][q][lane];
    merge8_keys(L, o);
  }
  __syncthreads();
  if (wave == 1)
#pragma unroll
    for (int q = 0; q < kBTopK; ++q) lists[1][q][lane] = L[q];
  __syncthreads();
  if (wave == 0 && j0 + lane < nact) {
    uint64_t o[kBTopK];
#pragma unroll
    for (int q = 0; q < kBTopK; ++q) o[q] = lists[1][q][lane];
    merge8_keys(L, o);
    uint64_t* out = partials + (static_cast<int64_t>(j0 + lane) * mtiles + blockIdx.x) * kBTopK;
#pragma unroll
    for (int q = 0; q < kBTopK; ++q) out[q] = L[q];
  }
}


template <int TI>
__global__ __launch_bounds__(kBCorrThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_bcorr(const uint16_t* __restrict__ psit,
                                                         int64_t ld, int64_t m,
                                                         const uint16_t* __restrict__ Rq,
                                                         int64_t ldq, const int* __restrict__ acts,
                                                         int64_t cap,
                                                         const BState* __restrict__ bs,
                                                         uint64_t* __restrict__ partials,
                                                         int mtiles, int par) {
  constexpr int TM = 16 * TI;
  const int nact = bs->n_active[par];
  const int* act = acts + par * cap;
  const int j0 = blockIdx.y * kBCorrTileB;
  if (j0 >= nact) return;  // workgroup-uniform
  const int lane = threadIdx.x % kWave;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform
  const int64_t m0 = static_cast<int64_t>(blockIdx.x) * TM;
  const int koff = 8 * (lane / 16);

  const uint16_t* arow[TI];
#pragma unroll
  for (int ti = 0; ti < TI; ++ti) {
    int64_t row = m0 + 16 * ti + (lane % 16);
    if (row > m - 1) row = m - 1;
    arow[ti] = psit + (row / 16) * 16 * ld + (row % 16) * 32 + koff;  // its tile row
  }
  const uint16_t* bcol[4];
#pragma unroll
  for (int tj = 0; tj < 4; ++tj) {
    int j = j0 + 16 * tj + (lane % 16);
    if (j > nact - 1) j = nact - 1;
    bcol[tj] = Rq + static_cast<int64_t>(act[j]) * ldq + koff;
  }
  v4f acc[TI][4];
#pragma unroll
  for (int ti = 0; ti < TI; ++ti)
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) acc[ti][tj] = v4f{0.f, 0.f, 0.f, 0.f};

  const int nsteps = static_cast<int>(ld / 32);
  // this wave's K-steps: wave, wave + 4, ...; `q` counts them
  const int nmine = nsteps > wave ? (nsteps - wave + kBCorrWaves - 1) / kBCorrWaves : 0;
  v8bf ra[kBPre][TI], rb[kBPre][4];
  auto load_step = [&](int slot, int q) {
    const int64_t k = static_cast<int64_t>(wave + q * kBCorrWaves) * 32;
#pragma unroll
    for (int ti = 0; ti < TI; ++ti)
      ra[slot][ti] = *reinterpret_cast<const v8bf*>(arow[ti] + k * 16);  // K chunk k / 32
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) rb[slot][tj] = *reinterpret_cast<const v8bf*>(bcol[tj] + k);
  };
  auto mma_step = [&](int slot) {
#pragma unroll
    for (int ti = 0; ti < TI; ++ti)
#pragma unroll
      for (int tj = 0; tj < 4; ++tj)
        acc[ti][tj] =
            __builtin_amdgcn_mfma_f32_16x16x32_bf16(ra[slot][ti], rb[slot][tj], acc[ti][tj], 0, 0, 0);
  };
  // the first kBPre steps (a step past the wave's last loads step 0 again,
  // which is valid memory and never used)
#pragma unroll
  for (int p = 0; p < kBPre; ++p) load_step(p, p < nmine ? p : 0);
  __builtin_amdgcn_sched_barrier(0);
  int q0 = 0;
  // steady state: every slot consumed is reloaded kBPre steps ahead
  for (; q0 + 2 * kBPre <= nmine; q0 += kBPre) {
#pragma unroll
    for (int p = 0; p < kBPre; ++p) {
      mma_step(p);
      load_step(p, q0 + p + kBPre);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // the last (fewer than 2 kBPre) steps
  for (; q0 < nmine; q0 += kBPre) {
#pragma unroll
    for (int p = 0; p < kBPre; ++p) {
      if (q0 + p < nmine) {
        mma_step(p);
        if (q0 + p + kBPre < nmine) load_step(p, q0 + p + kBPre);
      }
    }
  }

  // sum the four partial tiles: ((w0 + w2) + (w1 + w3)) into ctile[1]
  __shared__ float ctile[2][TM][kBCorrTileB + 1];
  __shared__ uint64_t lists[2][kBTopK][kBCorrTileB];
  auto store = [&](int slot) {
#pragma unroll
    for (int ti = 0; ti < TI; ++ti)
#pragma unroll
      for (int tj = 0; tj < 4; ++tj)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          ctile[slot][16 * ti + 4 * (lane / 16) + i][16 * tj + (lane % 16)] = acc[ti][tj][i];
  };
  auto add = [&](int slot) {
#pragma unroll
    for (int ti = 0; ti < TI; ++ti)
#pragma unroll
      for (int tj = 0; tj < 4; ++tj)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          acc[ti][tj][i] += ctile[slot][16 * ti + 4 * (lane / 16) + i][16 * tj + (lane % 16)];
  };
  if (wave >= 2) store(wave - 2);
  __syncthreads();
  if (wave < 2) add(wave);  // w0 + w2, w1 + w3
  __syncthreads();
  if (wave == 1) store(0);
  __syncthreads();
  if (wave == 0) {
    add(0);
    store(1);
  }
  __syncthreads();

  tile_top8<TM>(ctile[1], lists, m0, m, nact, j0, lane, wave, partials, mtiles);
}

// ---------------------------------------------------------------------------
// Product tile of 16 NW atoms x 64 signals with the residual operand staged
// in LDS (the form used while many signals are active): NW = 4 waves (64
// atoms, two workgroups per CU) or 8 waves (128 atoms, one workgroup per CU,
// a quarter less L2 -> L1 traffic per atom-signal product).  Wave w owns atom
// rows 16w .. 16w + 15 over all of K (4 MFMA 16x16 blocks per K-step, no
// reduction across waves); its dictionary operand comes straight from the
// tiled BF16 copy (1 KB per K-step, two register sets of one chunk each).
// The workgroup stages the 64 signals' residual rows chunk by chunk (kSChunk
// K elements, full 128-byte lines: 16 threads per row) into one of two LDS
// buffers while the MFMAs read the other; one barrier per chunk.  Used when
// ld is a multiple of 2 kSChunk.  Rows are padded by 16 bytes so that the
// 16 signal rows one operand read touches fall on distinct banks.  The
// residual buffers and the correlation tile share the LDS (the tile is
// written after the last chunk).  The epilogue is k_bcorr's.
constexpr int kSChunk = 128;                  // K elements per staged chunk (4 K-steps)
constexpr int kSRow = kSChunk + 8;            // LDS row stride in BF16 elements
template <int NW>
__global__ __launch_bounds__(NW * kWave) __attribute__((amdgpu_waves_per_eu(2))) void k_bcorr_s(
    const uint16_t* __restrict__ psit, int64_t ld, int64_t m, const uint16_t* Rq, int64_t ldq,
    const int* __restrict__ acts, int64_t cap, const BState* __restrict__ bs,
    uint64_t* __restrict__ partials, int mtiles, int par) {
  // Rq without __restrict__: its loads then stay where the memory clobber
  // below puts them (restrict-qualified loads count as invariant and move)
  static_assert(NW == 4 || NW == 8, "waves per workgroup");
  constexpr int NT = NW * kWave;
  constexpr int TM = 16 * NW;
  constexpr int SL = kBCorrTileB * kSChunk / 8 / NT;  // 16-byte staging loads per thread
  const int nact = bs->n_active[par];
  const int* act = acts + par * cap;
  const int j0 = blockIdx.y * kBCorrTileB;
  if (j0 >= nact) return;  // workgroup-uniform
  const int t = threadIdx.x;
  const int lane = t % kWave;
  const int wave = __builtin_amdgcn_readfirstlane(t / kWave);  // wave-uniform
  const int64_t m0 = static_cast<int64_t>(blockIdx.x) * TM;
  const int koff = 8 * (lane / 16);

  constexpr int kBufElems = kBCorrTileB * kSRow;
  constexpr int kBufBytes = 2 * kBufElems * 2;
  constexpr int kTileBytes = TM * (kBCorrTileB + 1) * 4;
  __shared__ __attribute__((aligned(16))) unsigned char smem[kBufBytes > kTileBytes ? kBufBytes
                                                                                   : kTileBytes];
  __shared__ uint64_t lists[2][kBTopK][kBCorrTileB];
  uint16_t(*bst)[kBufElems] = reinterpret_cast<uint16_t(*)[kBufElems]>(smem);
  float(*ctile)[kBCorrTileB + 1] = reinterpret_cast<float(*)[kBCorrTileB + 1]>(smem);

  // this wave's dictionary rows (rows past the last atom read the last one;
  // the epilogue skips them)
  int64_t row = m0 + 16 * wave + (lane % 16);
  if (row > m - 1) row = m - 1;
  const uint16_t* arow = psit + (row / 16) * 16 * ld + (row % 16) * 32 + koff;
  // this thread's share of the staging: row sig[q], 16 bytes at K offset soff
  const uint16_t* srow[SL];
  int sdst[SL];
#pragma unroll
  for (int q = 0; q < SL; ++q) {
    const int f = t + q * NT;
    const int sg = f / (kSChunk / 8);
    const int part = f % (kSChunk / 8);
    int j = j0 + sg;
    if (j > nact - 1) j = nact - 1;
    srow[q] = Rq + static_cast<int64_t>(act[j]) * ldq + 8 * part;
    sdst[q] = sg * kSRow + 8 * part;
  }
  const int nchunks = static_cast<int>(ld / kSChunk);

  v4f acc[4];
#pragma unroll
  for (int tj = 0; tj < 4; ++tj) acc[tj] = v4f{0.f, 0.f, 0.f, 0.f};
  constexpr int KS = kSChunk / 32;  // K-steps per chunk
  // two register sets of the dictionary operand, one chunk each
  v8bf ra[2][KS];
  auto load_a = [&](auto setc, int chunk) {
    constexpr int set = decltype(setc)::value;
#pragma unroll
    for (int kk = 0; kk < KS; ++kk)
      ra[set][kk] = *reinterpret_cast<const v8bf*>(
          arow + static_cast<int64_t>(chunk * KS + kk) * 32 * 16);
  };
  v4u sreg[SL];
  auto load_b = [&](int chunk) {
    const int64_t k0 = static_cast<int64_t>(chunk) * kSChunk;
#pragma unroll
    for (int q = 0; q < SL; ++q) sreg[q] = *reinterpret_cast<const v4u*>(srow[q] + k0);
  };
  auto store_b = [&](int buf) {
#pragma unroll
    for (int q = 0; q < SL; ++q) *reinterpret_cast<v4u*>(&bst[buf][sdst[q]]) = sreg[q];
  };
  // Chunk c (buffer and register set b = c mod 2): first request chunk c+1
  // (residual rows, then the dictionary operand into the other set), then
  // the MFMAs of chunk c from LDS and registers filled one chunk earlier, so
  // that no wait of chunk c covers a request of chunk c+1 made before it.
  auto chunk = [&](auto bc, int c) {
    constexpr int b = decltype(bc)::value;
    // unconditional (the last chunk requests itself again, unused): loads
    // under a branch would make the waits at the join cover them
    const int cn = c + 1 < nchunks ? c + 1 : c;
    load_b(cn);
    load_a(std::integral_constant<int, 1 - b>{}, cn);
    // keeps the requests here: without it the compiler moves the residual
    // loads down to their LDS store, where they would be waited for at once
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
      v8bf rb[4];
#pragma unroll
      for (int tj = 0; tj < 4; ++tj)
        rb[tj] = *reinterpret_cast<const v8bf*>(
            &bst[b][(16 * tj + (lane % 16)) * kSRow + 32 * kk + koff]);
#pragma unroll
      for (int tj = 0; tj < 4; ++tj)
        acc[tj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ra[b][kk], rb[tj], acc[tj], 0, 0, 0);
    }
    if (c + 1 < nchunks) store_b(1 - b);
    __syncthreads();
  };

  load_b(0);
  load_a(std::integral_constant<int, 0>{}, 0);
  store_b(0);
  __syncthreads();
  for (int c = 0; c < nchunks; c += 2) {  // nchunks is even (ld % 256 == 0)
    chunk(std::integral_constant<int, 0>{}, c);
    chunk(std::integral_constant<int, 1>{}, c + 1);
  }

#pragma unroll
  for (int tj = 0; tj < 4; ++tj)
#pragma unroll
    for (int i = 0; i < 4; ++i)
      ctile[16 * wave + 4 * (lane / 16) + i][16 * tj + (lane % 16)] = acc[tj][i];
  __syncthreads();
  tile_top8<TM>(ctile, lists, m0, m, nact, j0, lane, wave, partials, mtiles);
}

// ---------------------------------------------------------------------------
// Per-signal selection, FP32 re-scoring and update; one workgroup per
// position j of the round's list (list par, the product's), and one more,
// the grid's last, that compacts the list for the next round.  A signal that
// stopped in the previous round (still on this list) is skipped.  Stores
// the round's flag for position j: whether the signal goes on.
__global__ __launch_bounds__(kBSelThreads) void k_bselect(
    const float* __restrict__ psi32, int64_t ld, int64_t n, int64_t m,
    float* __restrict__ R32, uint16_t* __restrict__ Rq, int64_t ldq, float* __restrict__ X,
    int64_t ldx, BSlot* __restrict__ slots, int* __restrict__ acts, int* __restrict__ keep,
    int64_t cap, BState* __restrict__ bs, const uint64_t* __restrict__ partials, int mtiles,
    int par, int rescore_k, mp_trace tr) {
  const int nact = bs->n_active[par];
  int* flags_now = keep + par * cap;
  if (blockIdx.x == gridDim.x - 1) {
    // next round's list: the positions whose signal was still running after
    // the previous round (that round's flags, by the source position of each
    // entry in the previous list), with their source positions
    const int* flags_prev = keep + (par ^ 1) * cap;
    const int* src_now = keep + (2 + par) * cap;
    const int cnt = compact_list<kBSelThreads>(
        acts + par * cap, nact, [&](int jj) { return flags_prev[src_now[jj]] != 0; },
        acts + (par ^ 1) * cap, keep + (2 + (par ^ 1)) * cap);
    if (threadIdx.x == 0) bs->n_active[par ^ 1] = cnt;
    return;
  }
  const int j = blockIdx.x;
  if (j >= nact) return;
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  // this position's partial lists (the product wrote one descending list of
  // 8 keys per atom tile): the first group of this wave requested at once,
  // since it depends on the position only
  const uint64_t* pk = partials + static_cast<int64_t>(j) * mtiles * kBTopK;
  const int nkeys = mtiles * kBTopK;
  const int i0 = wave * 2 * kWave + lane;
  uint64_t ka = i0 < nkeys ? pk[i0] : 0ull;
  uint64_t kc = i0 + kWave < nkeys ? pk[i0 + kWave] : 0ull;
  const int b = acts[par * cap + j];
  BSlot* sl = slots + b;
  // the signal's state and r requested together; a signal that stopped in
  // the previous round (still on this list) is dropped after the merge
  const int was_done = sl->done;
  long long t0 = 0, tmax = 0;
  double thr = 0.0;
  if (threadIdx.x == 0) {
    t0 = sl->t;
    tmax = sl->max_iters;
    thr = sl->thr;
  }
  extern __shared__ v4f r_lds[];
  __shared__ uint64_t wl[kBSelWaves][kBTopK];
  __shared__ uint64_t resc[kBTopK];
  __shared__ double dred[kBSelWaves];
  float* r = R32 + static_cast<int64_t>(b) * ld;
  const int ld4 = static_cast<int>(ld / 4);
  for (int i = threadIdx.x; i < ld4; i += kBSelThreads) r_lds[i] = reinterpret_cast<const v4f*>(r)[i];

  // the signal's 8 best candidates: each wave merges 16 lists at a time
  // across its lanes and keeps a running top 8; then every wave merges the 8
  // waves' lists (the same result in each), so that wave q can take
  // candidate q without another barrier
  {
    uint64_t top = 0;
    for (int g = wave; g * 2 * kWave < nkeys; g += kBSelWaves) {
      if (g != wave) {
        const int i = g * 2 * kWave + lane;
        ka = i < nkeys ? pk[i] : 0ull;
        kc = i + kWave < nkeys ? pk[i + kWave] : 0ull;
      }
      top = merge_lane_lists8(top, top8_of_lists16(ka, kc, lane), lane);
    }
    if (lane < kBTopK) wl[wave][lane] = top;
  }
  if (was_done) {  // the same value in every thread
    if (threadIdx.x == 0) flags_now[j] = 0;
    return;
  }
  __syncthreads();
  static_assert(kBSelWaves * kBTopK == kWave, "one list per group of 8 lanes");
  const uint64_t t8 = top8_of_lists16(wl[lane / kBTopK][lane % kBTopK], 0ull, lane);
  // re-score in FP32, one candidate per wave (candidate q is lane q's key)
  for (int q = wave; q < rescore_k; q += kBSelWaves) {
    const uint64_t k =
        (static_cast<uint64_t>(static_cast<uint32_t>(__shfl(static_cast<int>(t8 >> 32), q)))
         << 32) |
        static_cast<uint32_t>(__shfl(static_cast<int>(t8 & 0xffffffffu), q));
    uint64_t rk = 0;
    if (k != 0) {
      const int idx = key_index(k);
      if (idx >= 0 && idx < m) {
        const float c32 = dot_column_f32<false>(
            reinterpret_cast<const v4f*>(psi32 + static_cast<int64_t>(idx) * ld), r_lds, ld4,
            lane);
        rk = make_key(c32, idx);
      }
    }
    if (lane == 0) resc[q] = rk;
  }
  __syncthreads();
  uint64_t best = 0;
  for (int q = 0; q < rescore_k; ++q) best = resc[q] > best ? resc[q] : best;
  const int idx = key_index(best);
  const float c = key_value(best);
  bool stop_now = false;
  if (best == 0 || idx < 0 || idx >= m) {
    stop_now = true;
    if (threadIdx.x == 0) {
      sl->done = 1;
      sl->reason = kStopInternal;
    }
  } else if (c == 0.0f) {
    stop_now = true;
    if (threadIdx.x == 0) {
      sl->done = 1;
      sl->reason = MP_STOP_STALLED;
    }
  }
  if (!stop_now) {
    // r -= c psi_idx from the LDS copy of r (padding rows stay 0), with its
    // BF16 copy, four elements per thread and step
    const v4f* colp = reinterpret_cast<const v4f*>(psi32 + static_cast<int64_t>(idx) * ld);
    v4f* r4 = reinterpret_cast<v4f*>(r);
    uint2* rq4 = reinterpret_cast<uint2*>(Rq + static_cast<int64_t>(b) * ldq);
    // this step's residual trace entry, if the trace asks for one (every
    // thread reads the step count: thread 0 rewrites it only after the
    // barriers of the norm below)
    float* rt = nullptr;
    if (tr.r) {
      const long long tt = sl->t;
      if (tt < tr.cap) rt = tr.r + (static_cast<int64_t>(b) * tr.cap + tt) * tr.ldr;
    }
    double s = 0.0;
    for (int i = threadIdx.x; i < ld4; i += kBSelThreads) {
      const v4f a = colp[i], rv = r_lds[i];
      v4f o;
      o.x = __builtin_fmaf(-c, a.x, rv.x);
      o.y = __builtin_fmaf(-c, a.y, rv.y);
      o.z = __builtin_fmaf(-c, a.z, rv.z);
      o.w = __builtin_fmaf(-c, a.w, rv.w);
      r4[i] = o;
      if (rt) trace_rows4(rt, i, n, o);
      rq4[i] = uint2{static_cast<uint32_t>(bf16_rne(o.x)) | (static_cast<uint32_t>(bf16_rne(o.y)) << 16),
                     static_cast<uint32_t>(bf16_rne(o.z)) | (static_cast<uint32_t>(bf16_rne(o.w)) << 16)};
      s += static_cast<double>(o.x) * o.x + static_cast<double>(o.y) * o.y +
           (static_cast<double>(o.z) * o.z + static_cast<double>(o.w) * o.w);
    }
    const double rr = block_sum<kBSelThreads>(s, dred);
    if (threadIdx.x == 0) {
      X[static_cast<int64_t>(b) * ldx + idx] += c;
      const long long t = t0;
      if (t < tr.cap) {
        const int64_t o = static_cast<int64_t>(b) * tr.cap + t;
        if (tr.idx) tr.idx[o] = idx;
        if (tr.coef) tr.coef[o] = c;
        if (tr.rr) tr.rr[o] = rr;
      }
      sl->t = t + 1;
      sl->rr = rr;
      if (!(rr > thr)) {
        sl->done = 1;
        sl->reason = MP_STOP_CONVERGED;
        stop_now = true;
      } else if (t + 1 >= tmax) {
        sl->done = 1;
        sl->reason = MP_STOP_MAX_ITERS;
        stop_now = true;
      }
    }
  }
  if (threadIdx.x == 0) flags_now[j] = stop_now ? 0 : 1;
}

// ---------------------------------------------------------------------------

hipError_t launch_tile_bf16(const float* psi, int64_t ld, int64_t m, uint16_t* out,
                            hipStream_t s) {
  k_tile_bf16<<<dim3(static_cast<unsigned>((m + 15) / 16)), dim3(256), 0, s>>>(psi, ld, m, out);
  return hipGetLastError();
}

hipError_t launch_binit(const float* Y, int64_t ldy, int64_t n, int64_t ld, float* X,
                        int64_t ldx, int64_t m, float* R32, uint16_t* Rq, int64_t ldq, BSlot* slots,
                        const long long* tcap, long long tcap_all, double eps, int nslots,
                        int* act, int* keep, int64_t cap, BState* bs, hipStream_t s) {
  k_binit<<<dim3(nslots), dim3(kBThreads), 0, s>>>(Y, ldy, n, ld, X, ldx, m, R32, Rq, ldq, slots,
                                                   tcap, tcap_all, eps);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_bcompact_init<<<dim3(1), dim3(kBThreads), 0, s>>>(nslots, slots, act, keep, cap, bs);
  return hipGetLastError();
}

// Atoms per product tile for a round expected to have `nact_hint` active
// signals: the more signals, the larger the tile (fewer dictionary re-reads
// per signal); the fewer, the smaller (more workgroups for the same work).
// The split-K tiles (32 and 16 atoms) sum each product in the same order,
// so they give the same values.  A larger tile yields to the next smaller
// one where its grid would leave CUs without a workgroup.
int bcorr_tile_m(int nact_hint, const BConfig& cf, int64_t ld, int64_t m, int num_cus) {
  const bool staged = ld % (2 * kSChunk) == 0;
  int t = 16;
  if (nact_hint > cf.atoms128_above && staged) t = 128;
  else if (nact_hint > cf.atoms64_above || nact_hint > cf.atoms128_above) t = 64;
  else if (nact_hint > cf.atoms32_above) t = 32;
  // a 128- or 64-atom tile only where its grid still gives every CU a
  // workgroup (a short dictionary: fewer atom tiles than CUs)
  const int64_t btiles = (nact_hint + kBCorrTileB - 1) / kBCorrTileB;
  while (t > 32 && (m + t - 1) / t * btiles < num_cus) t /= 2;
  return t;
}
int bcorr_mtiles(int64_t m, int tile_m) { return static_cast<int>((m + tile_m - 1) / tile_m); }

hipError_t launch_bround(const uint16_t* psit, const float* psi32, int64_t ld, int64_t n,
                         int64_t m, float* R32, uint16_t* Rq, int64_t ldq, float* X, int64_t ldx,
                         BSlot* slots, int* act, int* keep, int64_t cap, BState* bs,
                         uint64_t* partials, long long round, int nact_hint, const BConfig& cf,
                         int num_cus, int rescore_k, mp_trace tr, hipStream_t s, hipEvent_t e0,
                         hipEvent_t e1) {
  const int tile_m = bcorr_tile_m(nact_hint, cf, ld, m, num_cus);
  const int mtiles = bcorr_mtiles(m, tile_m);
  const int btiles = (nact_hint + kBCorrTileB - 1) / kBCorrTileB;  // >= the round's tiles
  const int par = static_cast<int>(round & 1);
  hipError_t e;
  if (e0 && (e = hipEventRecord(e0, s)) != hipSuccess) return e;
  const dim3 grid(mtiles, btiles > 0 ? btiles : 1);
  if (tile_m == 128)
    k_bcorr_s<8><<<grid, dim3(8 * kWave), 0, s>>>(psit, ld, m, Rq, ldq, act, cap, bs, partials,
                                                   mtiles, par);
  else if (tile_m == 64 && ld % (2 * kSChunk) == 0)
    k_bcorr_s<4><<<grid, dim3(4 * kWave), 0, s>>>(psit, ld, m, Rq, ldq, act, cap, bs, partials,
                                                   mtiles, par);
  else if (tile_m == 64)
    k_bcorr<4><<<grid, dim3(kBCorrThreads), 0, s>>>(psit, ld, m, Rq, ldq, act, cap, bs, partials,
                                                     mtiles, par);
  else if (tile_m == 32)
    k_bcorr<2><<<grid, dim3(kBCorrThreads), 0, s>>>(psit, ld, m, Rq, ldq, act, cap, bs, partials,
                                                     mtiles, par);
  else
    k_bcorr<1><<<grid, dim3(kBCorrThreads), 0, s>>>(psit, ld, m, Rq, ldq, act, cap, bs, partials,
                                                     mtiles, par);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (e1 && (e = hipEventRecord(e1, s)) != hipSuccess) return e;
  const size_t lds = static_cast<size_t>(ld) * sizeof(float);
  static bool big_lds = false;
  if (!big_lds && lds > 60 * 1024) {
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_bselect),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
    if (e != hipSuccess) return e;
    big_lds = true;
  }
  // one workgroup per list position, and the compacting one last
  k_bselect<<<dim3(nact_hint + 1), dim3(kBSelThreads), lds, s>>>(
      psi32, ld, n, m, R32, Rq, ldq, X, ldx, slots, act, keep, cap, bs, partials, mtiles, par,
      rescore_k, tr);
  return hipGetLastError();
}

}  // namespace mp
