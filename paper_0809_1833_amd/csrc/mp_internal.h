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
// Written by k_init and by the last workgroup of each iteration's launch.
struct alignas(64) DevState {
  double yy;            // ||y||^2
  double rr;            // ||r||^2 of the current residual
  double thr;           // eps^2 * ||y||^2: continue while rr > thr
  long long t;          // updates done
  long long max_iters;  // cap T
  int done;             // 1 once the run has stopped
  int reason;           // MP_STOP_* or kStopNonFinite
  unsigned arrive;      // workgroups of the current launch that have published a key
  int pad0;
  int pad[4];
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
hipError_t launch_mp_step_f32(const float* psi, int64_t ld, int64_t n, int64_t m, float* r,
                              const CorrGeom& g, uint64_t* keys, float* x, DevState* st,
                              mp_trace tr, hipStream_t s);

// ---- reduced-precision storage (k_lowp.hip) ---------------------------------
constexpr int kLpTopK = 8;  // candidates kept per pass and re-scored in FP32
hipError_t launch_quant_bf16(const float* psi, int64_t ld, int64_t m, uint16_t* out,
                             hipStream_t s);
hipError_t launch_quant_fp8(const float* psi, int64_t ld, int64_t m, uint8_t* out,
                            float* scales, hipStream_t s);
hipError_t launch_mp_step_lp(mp_dtype storage, const void* psiq, const float* scales,
                             const float* psi32, int64_t ld, int64_t n, int64_t m, float* r,
                             const CorrGeom& g, int rescore_k, uint64_t* keys, float* x,
                             DevState* st, mp_trace tr, hipStream_t s);

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
  uint64_t* partials = nullptr;  // key slots: kLpTopK per correlation workgroup
  mp::CorrGeom geom{};
  // profiling of the correlation kernel
  bool profiling = false;
  int prof_every = 1;            // time every prof_every-th launch
  std::vector<hipEvent_t> ev;    // 2 slots x 2 events x max chunk
  double prof_ms = 0.0;
  int64_t prof_launches = 0;
  int rescore_k = mp::kLpTopK;   // for the current decode
  std::string err;
};
