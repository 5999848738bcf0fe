// Internal declarations shared by the host API and the kernel files of libmp.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/mp.h"

namespace mp {

// Stop reason used internally for a non-finite y; the API maps it to MP_ENONFINITE.
constexpr int kStopNonFinite = -1;

// Solver state of one decode, resident in device memory for the whole run.
// Written only by the single-workgroup select/update kernels (and init).
struct alignas(64) DevState {
  double yy;            // ||y||^2
  double rr;            // ||r||^2 of the current residual
  double thr;           // eps^2 * ||y||^2: continue while rr > thr
  long long t;          // updates done
  long long max_iters;  // cap T
  int done;             // 1 once the run has stopped
  int reason;           // MP_STOP_* or kStopNonFinite
  int pad[6];
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
hipError_t launch_corr_f32(const float* psi, int64_t ld, int64_t m, const float* r,
                           const CorrGeom& g, uint64_t* partials, const DevState* st,
                           hipStream_t s);
hipError_t launch_select_update_f32(const uint64_t* partials, int np, const float* psi,
                                    int64_t ld, int64_t n, float* x, float* r, DevState* st,
                                    mp_trace tr, hipStream_t s);

}  // namespace mp

// The context behind the opaque mp_ctx handle.
struct mp_ctx {
  int device = 0;
  int num_cus = 0;
  int64_t n = 0, m = 0, ld = 0;  // ld: padded leading dimension of the owned copies
  mp_dtype storage = MP_F32;
  float* psi32 = nullptr;        // FP32 master, ld x m, zero padded rows n..ld-1
  void* psiq = nullptr;          // BF16 / FP8 copy (same layout), if any
  float* scales = nullptr;       // FP8 per-column scales
  // per-decode work buffers
  float* r_work = nullptr;       // ld floats, rows n..ld-1 stay zero
  mp::DevState* st = nullptr;    // device state
  mp::DevState* h_st = nullptr;  // pinned host mirror
  uint64_t* partials = nullptr;  // one key per correlation workgroup
  mp::CorrGeom geom{};
  // profiling of the correlation kernel
  bool profiling = false;
  std::vector<hipEvent_t> ev;    // 2 slots x 2 events x max chunk
  double prof_ms = 0.0;
  int64_t prof_launches = 0;
  std::string err;
};
