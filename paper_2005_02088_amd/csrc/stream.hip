// Attainable HBM bandwidth of a CU share: plain streaming kernels (fill, reduction,
// copy) on a CU-masked stream, timed on the device clock. They give the bandwidth
// roofline of a stage kernel confined to its share, and the ceiling of the
// device-global handoff (a writer on one share while a reader runs on another).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "internal.h"

namespace camelot {
namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
constexpr int kStreamUnroll = 8;
constexpr int kStreamWgPerCu = 2;

struct StreamArgs {
  const u32x4* src;
  u32x4* dst;
  int64_t n16;          // 16-byte words per pass
  int32_t reps;
  uint64_t* result;     // [0] first start (min), [1] last end (max), [2] checksum
};

__device__ __forceinline__ void stream_begin(const StreamArgs& a) {
  if (threadIdx.x == 0) atomicMin((unsigned long long*)&a.result[0], (unsigned long long)wall_clock64());
}

__device__ __forceinline__ void stream_end(const StreamArgs& a, uint32_t acc) {
  __syncthreads();
  if (threadIdx.x == 0) atomicMax((unsigned long long*)&a.result[1], (unsigned long long)wall_clock64());
  if (acc == 0x9E3779B1u) atomicAdd((unsigned long long*)&a.result[2], 1ull);   // keeps the loads live
}

// Each thread keeps kStreamUnroll independent 16-byte accesses in flight; the grid
// strides over the buffer in blocks of grid * 256 * kStreamUnroll words.
__global__ __launch_bounds__(kThreads) void stream_read(StreamArgs a) {
  stream_begin(a);
  const int64_t step = (int64_t)gridDim.x * kThreads;
  uint32_t acc = 0;
  for (int r = 0; r < a.reps; ++r) {
    int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    for (; i + (kStreamUnroll - 1) * step < a.n16; i += kStreamUnroll * step) {
      u32x4 v[kStreamUnroll];
#pragma unroll
      for (int u = 0; u < kStreamUnroll; ++u) v[u] = __builtin_nontemporal_load(a.src + i + u * step);
#pragma unroll
      for (int u = 0; u < kStreamUnroll; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    }
    for (; i < a.n16; i += step) {
      const u32x4 v = __builtin_nontemporal_load(a.src + i);
      acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
  }
  stream_end(a, acc);
}

__global__ __launch_bounds__(kThreads) void stream_write(StreamArgs a) {
  stream_begin(a);
  const int64_t step = (int64_t)gridDim.x * kThreads;
  for (int r = 0; r < a.reps; ++r) {
    const u32x4 v = (u32x4){(uint32_t)r, 1u, 2u, 3u};
    int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    for (; i + (kStreamUnroll - 1) * step < a.n16; i += kStreamUnroll * step) {
#pragma unroll
      for (int u = 0; u < kStreamUnroll; ++u) __builtin_nontemporal_store(v, a.dst + i + u * step);
    }
    for (; i < a.n16; i += step) __builtin_nontemporal_store(v, a.dst + i);
  }
  stream_end(a, 0);
}

__global__ __launch_bounds__(kThreads) void stream_copy(StreamArgs a) {
  stream_begin(a);
  const int64_t step = (int64_t)gridDim.x * kThreads;
  for (int r = 0; r < a.reps; ++r) {
    int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    for (; i + (kStreamUnroll - 1) * step < a.n16; i += kStreamUnroll * step) {
      u32x4 v[kStreamUnroll];
#pragma unroll
      for (int u = 0; u < kStreamUnroll; ++u) v[u] = __builtin_nontemporal_load(a.src + i + u * step);
#pragma unroll
      for (int u = 0; u < kStreamUnroll; ++u) __builtin_nontemporal_store(v[u], a.dst + i + u * step);
    }
    for (; i < a.n16; i += step) __builtin_nontemporal_store(__builtin_nontemporal_load(a.src + i), a.dst + i);
  }
  stream_end(a, 0);
}

}  // namespace
}  // namespace camelot

using namespace camelot;

extern "C" int32_t camelot_stream_bench(int32_t mode, int64_t bytes, int32_t n_cus, int32_t cu_offset, int32_t reps,
                                        double* out) {
  clear_error();
  if (!out) return fail(CAMELOT_EINVAL, "out is NULL");
  if (bytes < 16 || bytes % 16 != 0 || reps < 1) return fail(CAMELOT_EINVAL, "bytes must be a positive multiple of 16; reps >= 1");
  if (mode < CAMELOT_STREAM_READ || mode > CAMELOT_STREAM_SPLIT) return fail(CAMELOT_EINVAL, "unknown stream mode %d", mode);
  DevInfo dev;
  int32_t rc = dev_info(&dev);
  if (rc) return rc;
  const bool split = mode == CAMELOT_STREAM_SPLIT;
  if ((rc = check_share(n_cus, cu_offset, dev.n_cus))) return rc;
  if (split && (rc = check_share(n_cus, cu_offset + n_cus, dev.n_cus))) return rc;
  std::memset(out, 0, 3 * sizeof(double));
  hipStream_t s0, s1 = nullptr;
  if ((rc = cached_stream(cu_offset, n_cus, &s0))) return rc;
  if (split && (rc = cached_stream(cu_offset + n_cus, n_cus, &s1))) return rc;
  u32x4 *b0 = nullptr, *b1 = nullptr;
  uint64_t* res = nullptr;
  const bool two = mode == CAMELOT_STREAM_COPY || split;
  if ((rc = dmalloc(&b0, bytes)) || (two && (rc = dmalloc(&b1, bytes))) || (rc = dmalloc(&res, 64))) {
    dfree(b0);
    dfree(b1);
    return rc;
  }
  uint64_t init[8] = {~0ull, 0, 0, 0, 0, 0, 0, 0};
  rc = h2d(res, init, 64);
  // the buffers read hold defined values
  if (!rc) rc = dzero(b0, bytes);
  if (!rc && two) rc = dzero(b1, bytes);
  (void)hipStreamSynchronize(mem_stream());
  if (!rc) {
    StreamArgs a{b0, b1, bytes / 16, reps, res};
    const dim3 grid(kStreamWgPerCu * n_cus), block(kThreads);
    void* args[] = {(void*)&a};
    hipError_t e = hipSuccess;
    if (mode == CAMELOT_STREAM_READ) e = hipLaunchKernel((const void*)stream_read, grid, block, args, 0, s0);
    else if (mode == CAMELOT_STREAM_WRITE) {
      a.dst = b0;
      e = hipLaunchKernel((const void*)stream_write, grid, block, args, 0, s0);
    } else if (mode == CAMELOT_STREAM_COPY) e = hipLaunchKernel((const void*)stream_copy, grid, block, args, 0, s0);
    else {
      // writer on the first share, reader of the other buffer on the second
      StreamArgs w{nullptr, b1, bytes / 16, reps, res};
      void* wargs[] = {(void*)&w};
      e = hipLaunchKernel((const void*)stream_read, grid, block, args, 0, s1);
      if (e == hipSuccess) e = hipLaunchKernel((const void*)stream_write, grid, block, wargs, 0, s0);
    }
    if (e != hipSuccess) rc = fail(CAMELOT_EDEVICE, "stream kernel launch: %s", hipGetErrorString(e));
    if (hipStreamSynchronize(s0) != hipSuccess || (s1 && hipStreamSynchronize(s1) != hipSuccess))
      rc = rc ? rc : fail(CAMELOT_EDEVICE, "stream kernel failed");
  }
  uint64_t r[8] = {0};
  if (!rc) rc = d2h(r, res, 64);
  dfree(b0);
  dfree(b1);
  dfree(res);
  (void)hipStreamSynchronize(mem_stream());
  if (rc) return rc;
  const double moved = (double)bytes * reps * (two ? 2.0 : 1.0);
  out[0] = (double)(r[1] - r[0]) / (double)dev.wclk_hz;
  out[1] = moved;
  out[2] = out[0] > 0 ? moved / out[0] / 1e9 : 0.0;
  return CAMELOT_OK;
}
