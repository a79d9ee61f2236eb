// Standalone driver of the roofline measurement of the BF16 MLP stage (the dominant
// kernel of the speech pipeline): MLP 440-2048-2048-2048-4096 at a batch of 128
// rows on a CU share, through the library's one-shot stage kernel. A plain
// executable (no Python, no torch) so that a profiler can wrap it directly.
//
//   camelot_mlp_roofline <n_cus> <launches> <reps_per_launch>
//
// Prints one JSON line: the HIP-event time of every launch (on the stream the
// kernel runs on) and the mean time per batch. Weights and inputs are seeded
// pseudo-random values (their values do not change the work).
//
//   camelot_mlp_roofline copy <MiB>
//
// Runs a plain 16-byte-per-thread copy kernel over <MiB> MiB three times: the
// known-size reference against which hardware byte counters are scaled.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "camelot.h"

namespace {
uint64_t next(uint64_t& s) {  // SplitMix64 (Steele, Lea & Flood)
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
float unit(uint64_t& s) { return (float)((next(s) >> 40) * (1.0 / (1ull << 24)) * 2.0 - 1.0); }
uint16_t bf16_bits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__global__ void copy16(const uint4* __restrict__ src, uint4* __restrict__ dst, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

int run_copy(int mib) {
  const size_t bytes = (size_t)mib << 20, n = bytes / 16;
  void *a = nullptr, *b = nullptr;
  if (hipMalloc(&a, bytes) != hipSuccess || hipMalloc(&b, bytes) != hipSuccess) return 1;
  if (hipMemset(a, 1, bytes) != hipSuccess) return 1;
  for (int i = 0; i < 3; ++i) hipLaunchKernelGGL(copy16, dim3(4096), dim3(256), 0, 0, (const uint4*)a, (uint4*)b, n);
  if (hipDeviceSynchronize() != hipSuccess) return 1;
  std::printf("{\"copy_bytes\": %zu, \"launches\": 3}\n", bytes);
  hipFree(a);
  hipFree(b);
  return 0;
}

int die(const char* what) {
  std::fprintf(stderr, "%s: %s\n", what, camelot_last_error());
  return 1;
}
}  // namespace

int main(int argc, char** argv) {
  if (argc == 3 && std::strcmp(argv[1], "copy") == 0) return run_copy(std::atoi(argv[2]));
  if (argc != 4) {
    std::fprintf(stderr, "usage: %s <n_cus> <launches> <reps_per_launch>\n", argv[0]);
    return 2;
  }
  const int n_cus = std::atoi(argv[1]), launches = std::atoi(argv[2]), reps = std::atoi(argv[3]);
  if (n_cus < 8 || launches < 1 || reps < 1) return 2;
  const int dims[5] = {440, 2048, 2048, 2048, 4096};
  const int rows = 128;
  uint64_t seed = 12345;
  camelot_stage_desc d;
  std::memset(&d, 0, sizeof d);
  d.kind = CAMELOT_STAGE_MLP_BF16;
  d.n_layers = 4;
  std::vector<void*> bufs;
  for (int l = 0; l < 5; ++l) d.dims[l] = dims[l];
  for (int l = 0; l < 4; ++l) {
    const size_t n = (size_t)dims[l] * dims[l + 1];
    std::vector<uint16_t> w(n);
    const float scale = 1.0f / std::sqrt((float)dims[l]);
    for (auto& v : w) v = bf16_bits(unit(seed) * scale);
    void* p = nullptr;
    if (hipMalloc(&p, n * 2) != hipSuccess || hipMemcpy(p, w.data(), n * 2, hipMemcpyHostToDevice) != hipSuccess) {
      std::fprintf(stderr, "device allocation failed\n");
      return 1;
    }
    d.weights[l] = p;
    bufs.push_back(p);
  }
  std::vector<float> x((size_t)rows * dims[0]);
  for (auto& v : x) v = unit(seed);
  void *din = nullptr, *dout = nullptr;
  if (hipMalloc(&din, x.size() * 4) != hipSuccess || hipMalloc(&dout, (size_t)rows * dims[4] * 4) != hipSuccess ||
      hipMemcpy(din, x.data(), x.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
    std::fprintf(stderr, "device allocation failed\n");
    return 1;
  }
  double ns = 0, dns = 0;
  // one untimed launch first: the first launch of a kernel includes loading its code
  if (camelot_stage_run(&d, din, dout, rows, n_cus, 0, 1, &ns, &dns)) return die("warm-up");
  std::vector<double> per(launches);
  double sum = 0;
  for (int i = 0; i < launches; ++i) {
    if (camelot_stage_run(&d, din, dout, rows, n_cus, 0, reps, &ns, &dns)) return die("launch");
    per[i] = ns * reps / 1e3;  // microseconds per launch
    sum += ns;
  }
  std::printf("{\"n_cus\": %d, \"rows\": %d, \"reps_per_launch\": %d, \"launch_us\": [", n_cus, rows, reps);
  for (int i = 0; i < launches; ++i) std::printf("%s%.3f", i ? ", " : "", per[i]);
  std::printf("], \"ns_per_batch\": %.1f}\n", sum / launches);
  hipFree(din);
  hipFree(dout);
  for (void* p : bufs) hipFree(p);
  return 0;
}
