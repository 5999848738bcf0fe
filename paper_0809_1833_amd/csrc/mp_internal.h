// Internal declarations shared by the host API and the kernel files of libmp.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/mp.h"

namespace mp {

// Stop reasons used internally: a non-finite y (the API maps it to
// MP_ENONFINITE) and a selected index outside the dictionary, which a correct
// run never produces (MP_EDEVICE).
constexpr int kStopNonFinite = -1;
constexpr int kStopInternal = -2;

// Solver state of one decode, resident in device memory for the whole run.
// Written by k_init and by one workgroup of each step launch (workgroup 0 in
// the carried forms, the last to arrive in the OMP selection).
struct alignas(64) DevState {
  double yy;            // ||y||^2
  double rr;            // ||r||^2 of the current residual
  double thr;           // eps^2 * ||y||^2: continue while rr > thr
  long long t;          // updates done
  long long max_iters;  // cap T
  int done;             // 1 once the run has stopped
  int reason;           // MP_STOP_* or kStopNonFinite
  unsigned arrive;      // OMP selection: workgroups of the launch that have published a key
  int r_sel;            // reduced-precision decode: half of the residual buffer holding r
  int fail;             // persistent one-bit decode: set (atomic OR) by a workgroup whose
                        // wait gave up; overrides reason whatever was stored after it
  int pad[3];
};

// A candidate packed into one 64-bit key so that "larger key" means larger
// |c|, and among equal |c| the smaller column index:
//   bits 63..32  |c| as FP32 bits (sign cleared; NaN mapped to 0)
//   bits 31..1   0x7FFFFFFF - index
//   bit  0       sign of c
// The exact FP32 c and its index are recovered from the key.
__host__ __device__ inline uint64_t make_key(float c, int idx) {
  uint32_t u = __builtin_bit_cast(uint32_t, c);
  uint32_t ab = u & 0x7FFFFFFFu;
  if (ab > 0x7F800000u) ab = 0u;
  return (static_cast<uint64_t>(ab) << 32) |
         (static_cast<uint64_t>(0x7FFFFFFFu - static_cast<uint32_t>(idx)) << 1) |
         static_cast<uint64_t>(u >> 31);
}
__host__ __device__ inline int key_index(uint64_t k) {
  return static_cast<int>(0x7FFFFFFFu - (static_cast<uint32_t>(k) >> 1));
}
__host__ __device__ inline float key_value(uint64_t k) {
  uint32_t ab = static_cast<uint32_t>(k >> 32);
  uint32_t sg = static_cast<uint32_t>(k) & 1u;
  return __builtin_bit_cast(float, ab | (sg << 31));
}

// Column shares of the carried FP32 and FP64 passes.  The workgroups with the same
// blockIdx mod kBalGroups form a group (one XCD when workgroups go to the
// XCDs in turn) and take the same number of columns; each launch moves the
// groups' counts toward the column rates measured in the previous launch's
// pass.  Which workgroup streams a column does not change its correlation,
// so results do not depend on the shares.
constexpr int kBalGroups = 8;
constexpr int kBalMaxGrid = 1024;
struct BalState {  // device memory, per context, zeroed at creation
  int share[2][kBalGroups];      // columns per workgroup of each group, by launch parity
  unsigned dur[2][kBalMaxGrid];  // pass durations (wall-clock ticks), by launch parity
};

// Launch geometry of the FP32 correlation pass.
struct CorrGeom {
  int cols_per_wg;  // columns handled by one workgroup
  int grid;         // number of workgroups = number of partial keys
};

// ---- kernels of the FP32 single-signal path (k_f32.hip) -------------------
CorrGeom corr_f32_geometry(int64_t m, int num_cus);
hipError_t launch_norms(const float* psi, int64_t ld, int64_t n, int64_t m, double* norm2,
                        int* nonfinite, hipStream_t s);
hipError_t launch_init(const float* y, int64_t n, int64_t ld, float* x, int64_t m, float* r,
                       DevState* st, double eps, long long max_iters, hipStream_t s);
// ---- the static scratch of mp_solve_noalloc (mp_noalloc.hip) ---------------
// Layout: the decode state at 0, the residual double buffer (2 x ld floats,
// ld <= kNoAllocMaxLd) at kNoAllocR, the key slots (2 x grid x kLpTopK) at
// kNoAllocKeys, the column-share state at kNoAllocBal.
constexpr size_t kNoAllocScratchBytes = 256 * 1024;
constexpr int kNoAllocMaxDevices = 64;
constexpr int64_t kNoAllocMaxLd = 16384;
constexpr int64_t kNoAllocMaxKeys = 2 * 256 * 8;
constexpr size_t kNoAllocR = 256;
constexpr size_t kNoAllocKeys = kNoAllocR + 2 * kNoAllocMaxLd * sizeof(float);
constexpr size_t kNoAllocBal = kNoAllocKeys + kNoAllocMaxKeys * sizeof(uint64_t);
// The scratch's device address on `device` (which must be current), looked
// up once per device and kept.
hipError_t noalloc_scratch(int device, void** out);

// Small dictionaries (every workgroup's share of the columns in LDS): the
// whole FP32 decode in one launch.  small_geometry gives grid 0 where it
// does not apply.  rbuf: 2 x ld floats (r = y in half 0 from the init
// kernel; r after the last step in half 1).  slots: small_slot_words()
// words (two halves of one 2-word record per wave of every workgroup),
// zeroed at creation and whenever the epoch wraps.
CorrGeom small_geometry(int64_t ld, int64_t m, int num_cus);
hipError_t launch_f32_small(const float* psi, int64_t ld, int64_t n, int64_t m, float* rbuf,
                            const CorrGeom& g, unsigned long long* slots, unsigned epoch,
                            long long max_iters, float* x, DevState* st, mp_trace tr,
                            hipStream_t s);
unsigned small_epoch_mod();
int small_slot_words();

// n floats of the residual half st->r_sel names (rbuf: 2 x ld) into r.
hipError_t launch_copy_selected(const float* rbuf, int64_t ld, int64_t n, const DevState* st,
                                float* r, hipStream_t s);
// Launch k of an FP32 decode: step k (k >= 1) and pass k+1.  rbuf: 2 x ld
// floats (r in half k mod 2); keys: 2 halves x one per workgroup.  The stop
// threshold is read from st (set by the init kernel).
hipError_t launch_mp_step_f32(const float* psi, int64_t ld, int64_t n, int64_t m, float* rbuf,
                              const CorrGeom& g, uint64_t* keys, BalState* bal, long long k,
                              long long max_iters, float* x, DevState* st, mp_trace tr,
                              hipStream_t s);

// ---- kernels of the FP64 single-signal path (k_f64.hip) ---------------------
hipError_t launch_norms_f64(const double* psi, int64_t ld, int64_t n, int64_t m, double* norm2,
                            hipStream_t s);
hipError_t launch_init_f64(const double* y, int64_t n, int64_t ld, double* x, int64_t m,
                           double* r, DevState* st, double eps, long long max_iters,
                           hipStream_t s);
// Launch k of an FP64 decode: step k (k >= 1) and pass k+1.  rbuf: 2 x ld
// doubles (r in half k mod 2); keys: 2 halves x two words per workgroup.
hipError_t launch_mp_step_f64(const double* psi, int64_t ld, int64_t n, int64_t m, double* rbuf,
                              const CorrGeom& g, uint64_t* keys, BalState* bal, long long k,
                              long long max_iters, double thr, double* x, DevState* st,
                              mp_trace_f64 tr, hipStream_t s);

// ---- sign-bit Bernoulli dictionary (k_sign.hip) ------------------------------
// 16-byte chunks of a column each lane reads (1 for n <= 8192, 2 above).
int sign_chunks_per_lane(int64_t n);
CorrGeom sign_geometry(int64_t n, int64_t m, int num_cus);

// Step records of the persistent one-bit decode: kSignSlotWords arrays of
// 2 x grid 64-bit words (word q of workgroup g for steps of parity p at
// (q * 2 + p) * grid + g), each word a 32-bit tag over 32 bits of payload
// (the best key's two high halves, its low word, the partial ||r||^2's two
// halves); the tag is ((epoch mod 4096) << 20) | ((step + 1) mod 2^20) with
// epoch mod 4096 never 0, so the zeroed words match no step.
constexpr int kSignSlotWords = 5;
constexpr unsigned kSignEpochMod = 4096;
// Whether the persistent one-bit decode can hold this geometry (one
// workgroup per CU, the share's bits in LDS, rows of r in registers).
bool sign_persist_fits(int64_t n, int64_t m, int64_t ld, int64_t ws, const CorrGeom& g,
                       int num_cus);
// Whether the device keeps `g.grid` persistent workgroups resident at once
// (sets the kernel's LDS limit; false if it cannot).
bool sign_persist_resident(int64_t n, int64_t ws, const CorrGeom& g, int num_cus);
hipError_t launch_sign_persist(const uint32_t* bits, int64_t ws, int64_t n, int64_t m, int64_t ld,
                               const double* c64, double* r64, float* r32, const CorrGeom& g,
                               unsigned long long* slots, unsigned epoch, long long max_iters,
                               double thr, float* x, DevState* st, mp_trace tr, hipStream_t s);
// Packed input (ldw words per column) -> ws words per column, rows >= n cleared.
hipError_t launch_copy_signs(const uint32_t* in, int64_t ldw, int64_t n, int64_t m, int64_t ws,
                             uint32_t* out, hipStream_t s);
// c(0) = Psi^T y and r = y, both FP64 (c64: m, r64: ld doubles).
hipError_t launch_sign_c0(const uint32_t* bits, int64_t ws, int64_t n, int64_t m, const float* y,
                          int64_t ld, double* c64, double* r64, hipStream_t s);
// Launch k of a decode: stop test for the k-1 steps taken, step k, the keys
// of the next.  keys: 2 halves x 2 words x grid; rrp: 2 halves x grid.
hipError_t launch_mp_step_sign(const uint32_t* bits, int64_t ws, int64_t n, int64_t m, int64_t ld,
                               double* c64, double* r64, float* r32, double* rrp,
                               const CorrGeom& g, uint64_t* keys, long long k, long long max_iters,
                               double thr, float* x, DevState* st, mp_trace tr, hipStream_t s);

// ---- Orthogonal Matching Pursuit, FP32 (k_omp.hip) --------------------------
struct OmpState {           // the atom selected in the current iteration
  int sel;
  float c;                  // its correlation <r, psi_sel>
  int pad[2];
};
struct OmpBufs {            // work buffers of one OMP decode (context-owned)
  int64_t tq = 0;           // capacity: atoms (rows of q, order of R)
  float* q = nullptr;       // tq x ld: orthonormal basis of the selected atoms
  float* rmat = nullptr;    // tq x tq column-major upper triangle R (Psi_S = Q R)
  double* z = nullptr;      // tq: coordinates of y on q_0..q_{t-1}
  int* sel = nullptr;       // tq: selected atoms in order
  unsigned char* in_s = nullptr;  // m flags: atom already selected
  float* w = nullptr;       // ld: the vector being orthogonalised
  float* h1 = nullptr;      // tq: Q^T psi_i (first Gram-Schmidt pass)
  float* h2 = nullptr;      // tq: Q^T w (second pass)
  float* hp = nullptr;      // tq x kOmpProjSlices: the projections by slice of rows
  double* part = nullptr;   // ld / 64: per-workgroup sums of w^2
  OmpState* os = nullptr;
};
// Slices of rows the projections of an OMP iteration are split into.
constexpr int kOmpProjSlices = 8;
// One OMP iteration (five launches); t_bound >= the number of atoms selected
// so far (sizes the projection grid).  e0/e1 time the selection pass.
hipError_t launch_omp_iteration(const float* psi, int64_t ld, int64_t n, int64_t m, float* r,
                                const CorrGeom& g, uint64_t* keys, DevState* st, OmpBufs& b,
                                long long t_bound, mp_trace tr, hipStream_t s, hipEvent_t e0,
                                hipEvent_t e1);
hipError_t launch_omp_solve(const OmpBufs& b, const DevState* st, float* x, hipStream_t s);

// ---- batched decode against one dictionary (k_batched.hip) ------------------
// Per-signal state; written only by the workgroup handling that signal.
struct BSlot {
  double yy, rr, thr;
  long long t, max_iters;
  int done, reason;
};
// Round state.  Round r's product and select run over active list r mod 2
// (n_active[r mod 2] positions); the select also writes list (r+1) mod 2 for
// the next round.
struct BState {
  int n_active[2];
  int pad[2];
};
// The BF16 dictionary in the product's 16-atom x 32-element tiles
// (round_up(m, 16) x ld elements).
hipError_t launch_tile_bf16(const float* psi, int64_t ld, int64_t m, uint16_t* out,
                            hipStream_t s);
hipError_t launch_binit(const float* Y, int64_t ldy, int64_t n, int64_t ld, float* X,
                        int64_t ldx, int64_t m, float* R32, uint16_t* Rq, int64_t ldq, BSlot* slots,
                        const long long* tcap, long long tcap_all, double eps, int nslots,
                        int* act, int* keep, int64_t cap, BState* bs, hipStream_t s);
// Product tile by the number of active signals: 128 atoms (eight waves)
// while more than atoms128_above are active, 64 atoms while more than
// atoms64_above, 32 while more than atoms32_above, else 16; the two staged
// forms need ld % 256 == 0 (otherwise 64 atoms without staging), and a 128-
// or 64-atom tile yields to the next smaller one where its grid would have
// fewer workgroups than the device has CUs.  Chosen by the autotuner.
struct BConfig {
  int atoms128_above;
  int atoms64_above;
  int atoms32_above;
};
// By default no 128-atom tile (on N=2048, M=8192, B=256 it made the decode
// slower at every switch point tried: 46.4 against 44.4 ms) and no 16-atom
// tile.
constexpr BConfig kBConfigDefault{0x7fffffff, 96, 0};
constexpr int kBTileMinAtoms = 16;  // the smallest tile, which has the most partial lists
int bcorr_tile_m(int nact_hint, const BConfig& cf, int64_t ld, int64_t m, int num_cus);
int bcorr_mtiles(int64_t m, int tile_m);
// Round `round` (0, 1, ...).  nact_hint >= the number of active signals (the
// host's last reading; the count only decreases): it sizes the grids and
// picks the tile.  act: two lists of cap slots; keep: 4 x cap ints (the
// flags of rounds of parity 0 and 1, then the source positions of lists 0
// and 1).
hipError_t launch_bround(const uint16_t* psit, const float* psi32, int64_t ld, int64_t n,
                         int64_t m, float* R32, uint16_t* Rq, int64_t ldq, float* X, int64_t ldx,
                         BSlot* slots, int* act, int* keep, int64_t cap, BState* bs,
                         uint64_t* partials, long long round, int nact_hint, const BConfig& cf,
                         int num_cus, int rescore_k, mp_trace tr, hipStream_t s, hipEvent_t e0,
                         hipEvent_t e1);

// ---- many independent instances (k_ragged.hip) -------------------------------
struct RInst {             // one instance, device-resident descriptor
  const float* psi32;      // ld x m FP32 copy (zero padded rows)
  const uint16_t* psib;    // ld x m BF16 copy, or null
  int64_t n, m, ld;
  int64_t y_off, x_off;    // offsets of the instance in the packed Y / R and X
};
struct RResult {
  long long t;
  double yy, rr;
  int reason, pad;
};
struct RQueue {
  unsigned next;           // next position of the work list to take
  int fail;                // set (atomic OR) when a wait between the parts of an instance gave up
};
// One entry of the ragged work list: part `part` of `parts` of instance `id`
// (columns [part m / parts, (part + 1) m / parts)); the parts of one instance
// are consecutive in the list and exchange their candidates through record
// slot `slot` every step (slot < 0 when parts == 1).
struct RItem {
  int id, part, parts, slot;
};
constexpr int kRaggedMaxParts = 8;
constexpr int kRaggedRecWords = 16;  // words of one part's record: 8 keys, 2 words each
struct RConfig {           // launch shape, chosen by the autotuner
  int threads;             // workgroup size: 256, 512 or 1024
  int cols_per_wave;       // columns a wave streams at once: 1, 2 or 4
  int wgs_per_cu;          // persistent workgroups per CU
  int split;               // most parts an instance is cut into: 1 .. kRaggedMaxParts
};
bool ragged_config_valid(const RConfig& cf, bool lp);
// slots: nslots x 2 x kRaggedMaxParts x kRaggedRecWords words (cleared by the
// launch before the decode)
hipError_t launch_ragged(const RConfig& cf, bool lp, int grid, size_t lds, const RInst* inst,
                         const RItem* items, int nitems, const float* Y, float* X, float* R,
                         const long long* caps, long long cap_all, double eps, int rescore_k,
                         RResult* res, RQueue* q, unsigned long long* slots, int nslots,
                         long long spin_limit, mp_trace tr, hipStream_t s);

// ---- reduced-precision storage (k_lowp.hip) ---------------------------------
constexpr int kLpTopK = 8;  // candidates kept per pass and re-scored in FP32
hipError_t launch_quant_bf16(const float* psi, int64_t ld, int64_t m, uint16_t* out,
                             hipStream_t s);
hipError_t launch_quant_fp8(const float* psi, int64_t ld, int64_t m, uint8_t* out,
                            float* scales, hipStream_t s);
// Launch k of a reduced-precision decode: step k (k >= 1) and pass k+1.
// rbuf: 2 x ld floats (r in half k mod 2); keys: 2 halves x 8 per workgroup.
hipError_t launch_mp_step_lp(mp_dtype storage, const void* psiq, const float* scales,
                             const float* psi32, int64_t ld, int64_t n, int64_t m, float* rbuf,
                             const CorrGeom& g, int rescore_k, uint64_t* keys, long long k,
                             long long max_iters, float* x, DevState* st,
                             mp_trace tr, hipStream_t s);

}  // namespace mp

// The context behind the opaque mp_ctx handle.
struct mp_ctx {
  int device = 0;
  int num_cus = 0;
  int64_t n = 0, m = 0, ld = 0;  // ld: padded leading dimension of the owned copies
  mp_dtype storage = MP_F32;
  float* psi32 = nullptr;        // FP32 master, ld x m, zero padded rows n..ld-1
  double* psi64 = nullptr;       // MP_F64 storage: the FP64 dictionary (same layout)
  double* r64_work = nullptr;    // MP_F64 storage: ld doubles, rows n..ld-1 stay zero
  void* psiq = nullptr;          // BF16 / FP8 copy (same layout), if any
  uint32_t* psis = nullptr;      // MP_SIGN1 storage: sign bits, sign_ws words per column
  int64_t sign_ws = 0;           // words per column (ceil(n/32) rounded up to 4)
  double* sign_c64 = nullptr;    // MP_SIGN1: the carried correlations, m doubles
  double* sign_r64 = nullptr;    // MP_SIGN1: r in FP64, ld doubles
  double* sign_rrp = nullptr;    // MP_SIGN1: per-workgroup partial ||r||^2, 2 x grid
  unsigned long long* sign_slots = nullptr;  // MP_SIGN1 persistent decode: step records
  unsigned sign_epoch = 0;       // MP_SIGN1 persistent decode: tag epoch of the last decode
  bool sign_persist = false;     // MP_SIGN1: the persistent decode fits this device
  float* scales = nullptr;       // FP8 per-column scales
  // per-decode work buffers
  float* r_work = nullptr;       // ld floats, rows n..ld-1 stay zero
  mp::DevState* st = nullptr;    // device state
  mp::DevState* h_st = nullptr;  // pinned: host mirror, then two chunk-state slots
  hipEvent_t done_ev[2] = {nullptr, nullptr};  // the chunk-state copies done
  // a stream-ordered decode (MP_SOLVE_ASYNC): its state is copied into
  // h_st[0], then async_ev is recorded; collected by mp_solve_result
  hipEvent_t async_ev = nullptr;
  bool async_pending = false;
  int async_persistent = 0;
  uint64_t* partials = nullptr;  // key slots: kLpTopK per correlation workgroup
  mp::BalState* bal = nullptr;   // column shares and pass timings (FP32, FP64 passes)
  mp::CorrGeom geom{};
  mp::CorrGeom small{};          // MP_F32: the one-launch decode's shape (grid 0: not used)
  unsigned long long* small_slots = nullptr;  // its step records
  unsigned small_epoch = 0;      // tag epoch of its last decode
  // profiling of the correlation kernel
  bool profiling = false;
  int prof_every = 1;            // time every prof_every-th launch
  std::vector<hipEvent_t> ev;    // 2 slots x 2 events x max chunk
  double prof_ms = 0.0;
  int64_t prof_launches = 0;
  int rescore_k = mp::kLpTopK;   // for the current decode
  // batched decode: BF16 dictionary in product tiles and per-signal buffers
  // (grown on demand)
  uint16_t* psibt = nullptr;     // round_up(m, 16) x ld BF16, 16 x 32 tiles
  int64_t bcap = 0;              // signal slots allocated
  int64_t ldq = 0;               // leading dimension of b_rq: ld + 32
  float* b_r32 = nullptr;        // bcap x ld
  uint16_t* b_rq = nullptr;      // bcap x ldq
  mp::BSlot* b_slots = nullptr;
  mp::BSlot* h_slots = nullptr;  // pinned
  int* b_act = nullptr;          // 2 x bcap
  mp::BState* b_state = nullptr;
  mp::BState* h_bstate = nullptr;  // pinned, 2 entries
  uint64_t* b_partials = nullptr;  // bcap x mtiles x 8
  int* b_keep = nullptr;           // 4 x bcap: round flags (2 x), list source positions (2 x)
  long long* b_tcap = nullptr;     // bcap
  mp::BConfig b_cfg = mp::kBConfigDefault;  // product tile by active count
  // ragged contexts (mp_create_ragged): many instances, each its own dictionary
  bool ragged = false;
  int64_t r_count = 0;
  int64_t r_sum_n = 0, r_sum_m = 0, r_max_ld = 0;
  float* r_psi32 = nullptr;        // all instances' FP32 copies, packed
  uint16_t* r_psib = nullptr;      // all BF16 copies, packed (MP_BF16 storage)
  mp::RInst* r_inst = nullptr;     // device descriptors
  mp::RItem* r_items = nullptr;    // device: the work list (room for count x kRaggedMaxParts)
  unsigned long long* r_slots = nullptr;  // device: the split instances' step records
  int r_nitems = 0, r_nslots = 0;  // the work list uploaded for r_items_cfg
  mp::RConfig r_items_cfg{0, 0, 0, 0};
  std::vector<int> r_order;        // host: instance ids, most work first
  std::vector<double> r_est;       // host: work estimate of each instance
  long long* r_caps = nullptr;     // device: per-instance caps
  mp::RResult* r_res = nullptr;    // device results
  mp::RResult* h_rres = nullptr;   // pinned host copy
  mp::RQueue* h_rq = nullptr;      // pinned host copy of the queue (its fail word)
  mp::RQueue* r_queue = nullptr;
  mp::RConfig r_cfg{1024, 2, 1, 2};
  std::vector<int64_t> r_n, r_m;   // host copies of the sizes
  // the solve captured as a graph (replayed while its arguments are unchanged)
  hipStream_t r_cap_stream = nullptr;
  hipGraphExec_t r_graph = nullptr;
  std::vector<unsigned char> r_graph_key;
  // OMP decode buffers (grown on demand)
  mp::OmpBufs omp;
  std::string err;
};
