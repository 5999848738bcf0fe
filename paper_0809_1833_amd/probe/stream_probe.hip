// Streaming-bandwidth probe for MI355X: how fast can a kernel read (or copy)
// HBM with the access patterns the decoder uses?  Also the copy kernel of
// known size used to calibrate the FETCH_SIZE / WRITE_SIZE counters.
//
//   stream_probe read  <MiB> <reps>   grid-stride 16-byte non-temporal reads
//   stream_probe chunk <MiB> <reps>   each workgroup reads one contiguous chunk
//   stream_probe copy  <MiB> <reps>   16-byte loads and stores, dst = src
//
// Prints one JSON line per run: bytes moved per launch and GB/s (mean over
// the timed launches, HIP events).
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef float v4f __attribute__((ext_vector_type(4)));

#define CHECK(x)                                                              \
  do {                                                                        \
    hipError_t e_ = (x);                                                      \
    if (e_ != hipSuccess) {                                                   \
      fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));                 \
      exit(1);                                                                \
    }                                                                         \
  } while (0)

constexpr int kThreads = 256;
constexpr int kUnroll = 8;

__global__ __launch_bounds__(kThreads) void k_read(const v4f* __restrict__ src, size_t n16,
                                                   float* __restrict__ sink) {
  const size_t stride = static_cast<size_t>(gridDim.x) * kThreads;
  size_t i = static_cast<size_t>(blockIdx.x) * kThreads + threadIdx.x;
  float acc = 0.f;
  for (; i + stride * (kUnroll - 1) < n16; i += stride * kUnroll) {
    v4f a[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) a[u] = __builtin_nontemporal_load(src + i + stride * u);
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) acc += a[u].x + a[u].y + a[u].z + a[u].w;
  }
  for (; i < n16; i += stride) {
    v4f a = __builtin_nontemporal_load(src + i);
    acc += a.x + a.y + a.z + a.w;
  }
  sink[static_cast<size_t>(blockIdx.x) * kThreads + threadIdx.x] = acc;
}

__global__ __launch_bounds__(kThreads) void k_chunk(const v4f* __restrict__ src, size_t n16,
                                                    size_t per_block, float* __restrict__ sink) {
  const size_t b0 = static_cast<size_t>(blockIdx.x) * per_block;
  size_t b1 = b0 + per_block;
  if (b1 > n16) b1 = n16;
  float acc = 0.f;
  size_t i = b0 + threadIdx.x;
  for (; i + kThreads * (kUnroll - 1) < b1; i += kThreads * kUnroll) {
    v4f a[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) a[u] = __builtin_nontemporal_load(src + i + kThreads * u);
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) acc += a[u].x + a[u].y + a[u].z + a[u].w;
  }
  for (; i < b1; i += kThreads) {
    v4f a = __builtin_nontemporal_load(src + i);
    acc += a.x + a.y + a.z + a.w;
  }
  sink[static_cast<size_t>(blockIdx.x) * kThreads + threadIdx.x] = acc;
}

__global__ __launch_bounds__(kThreads) void k_copy(const v4f* __restrict__ src,
                                                   v4f* __restrict__ dst, size_t n16) {
  const size_t stride = static_cast<size_t>(gridDim.x) * kThreads;
  for (size_t i = static_cast<size_t>(blockIdx.x) * kThreads + threadIdx.x; i < n16; i += stride)
    dst[i] = src[i];
}

int main(int argc, char** argv) {
  if (argc < 4) {
    fprintf(stderr, "usage: %s read|chunk|copy <MiB> <reps> [blocks]\n", argv[0]);
    return 2;
  }
  const char* mode = argv[1];
  const size_t bytes = static_cast<size_t>(atol(argv[2])) << 20;
  const int reps = atoi(argv[3]);
  hipDeviceProp_t prop;
  CHECK(hipGetDeviceProperties(&prop, 0));
  int blocks = argc > 4 ? atoi(argv[4]) : prop.multiProcessorCount * 8;
  const size_t n16 = bytes / 16;
  v4f *src = nullptr, *dst = nullptr;
  float* sink = nullptr;
  CHECK(hipMalloc(&src, bytes));
  CHECK(hipMemset(src, 0, bytes));
  const bool copy = strcmp(mode, "copy") == 0;
  const bool chunk = strcmp(mode, "chunk") == 0;
  if (copy) CHECK(hipMalloc(&dst, bytes));
  size_t per_block = (n16 + blocks - 1) / blocks;
  CHECK(hipMalloc(&sink, sizeof(float) * static_cast<size_t>(blocks) * kThreads));
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  auto launch = [&]() {
    if (copy) k_copy<<<blocks, kThreads>>>(src, dst, n16);
    else if (chunk) k_chunk<<<blocks, kThreads>>>(src, n16, per_block, sink);
    else k_read<<<blocks, kThreads>>>(src, n16, sink);
  };
  launch();  // warm-up
  CHECK(hipDeviceSynchronize());
  float total = 0.f;
  for (int r = 0; r < reps; ++r) {
    CHECK(hipEventRecord(e0, 0));
    launch();
    CHECK(hipEventRecord(e1, 0));
    CHECK(hipEventSynchronize(e1));
    float ms = 0.f;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    total += ms;
  }
  CHECK(hipGetLastError());
  const double moved = static_cast<double>(bytes) * (copy ? 2.0 : 1.0);
  const double avg = total / reps;
  printf("{\"mode\": \"%s\", \"bytes_read\": %zu, \"bytes_written\": %zu, \"blocks\": %d, "
         "\"avg_ms\": %.4f, \"gbps\": %.1f}\n",
         mode, bytes, copy ? bytes : 0, blocks, avg, moved / (avg * 1e-3) / 1e9);
  CHECK(hipFree(src));
  if (dst) CHECK(hipFree(dst));
  CHECK(hipFree(sink));
  return 0;
}
