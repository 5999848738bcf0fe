// Wave64 / workgroup reductions used by the decoder's kernels (gfx950).
//
// All reductions combine values in a fixed pattern (xor butterflies inside a
// wave, then the per-wave results in wave order), so a given launch shape
// always produces bit-identical results.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mp {

constexpr int kWave = 64;

__device__ inline float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ inline uint64_t wave_max(uint64_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    uint64_t o = __shfl_xor(static_cast<unsigned long long>(v), off, kWave);
    v = o > v ? o : v;
  }
  return v;
}

// Workgroup-wide sum of a double; every thread receives the result.
// `red` must hold NT/64 doubles of LDS.
template <int NT>
__device__ inline double block_sum(double v, double* red) {
  constexpr int NW = NT / kWave;
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  v = wave_sum(v);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = lane < NW ? red[lane] : 0.0;
  s = wave_sum(s);
  __syncthreads();  // red may be reused by the caller
  return s;
}

// Workgroup-wide max of a 64-bit key; every thread receives the result.
template <int NT>
__device__ inline uint64_t block_max(uint64_t v, uint64_t* red) {
  constexpr int NW = NT / kWave;
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  v = wave_max(v);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  uint64_t s = lane < NW ? red[lane] : 0ull;
  s = wave_max(s);
  __syncthreads();
  return s;
}

}  // namespace mp
