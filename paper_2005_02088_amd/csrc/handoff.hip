// Device-global handoff benchmark (the global-memory communication of Section VI-B
// measured on its own): a persistent producer grid writes ring slots and rings a
// doorbell per (slot, workgroup) channel; a persistent consumer grid on other CUs
// waits on each doorbell, folds every 32-bit word of the chunk into a checksum and
// frees the slot. Producer workgroup j and consumer workgroup j own the same chunk
// of every slot, so the channels are independent (no grid barrier). All waits are
// bounded by spin_ticks. The producer writes its chunk through to the device's point
// of coherence (cache policy nt sc1) and every wave waits for its stores before the
// workgroup barrier, so thread 0 rings the doorbell right after it (with plain stores
// and one release by thread 0, a reader on another XCD sometimes saw old data behind
// the new doorbell).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"

namespace camelot {

// Pattern word w of slot s: (s * 0x9E3779B1) xor w (32-bit arithmetic).
__device__ __forceinline__ uint32_t pattern(uint64_t s, uint32_t w) {
  return ((uint32_t)s * 0x9E3779B1u) ^ w;
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
constexpr int kUnroll = 8;
constexpr int kStreamThrough = 18;     // cache policy nt sc1
constexpr int64_t kStep = (int64_t)kThreads * 16;

__device__ __forceinline__ u32x4 pattern4(uint64_t s, uint32_t w) {
  return (u32x4){pattern(s, w), pattern(s, w + 1), pattern(s, w + 2), pattern(s, w + 3)};
}

__device__ __forceinline__ bool wait_eq(const uint32_t* p, uint32_t want, int64_t spin_ticks, uint64_t* err) {
  const uint64_t t0 = now_ticks();
  while (__hip_atomic_load(const_cast<uint32_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != want) {
    if ((int64_t)(now_ticks() - t0) > spin_ticks) {
      __hip_atomic_store(err, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
    __builtin_amdgcn_s_sleep(1);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return true;
}

extern "C" __global__ __launch_bounds__(kThreads, kMinWgPerCuResident) void camelot_handoff_producer(HandoffArgs a) {
  __shared__ int s_ok;
  const int j = blockIdx.x, nwg = gridDim.x, tid = threadIdx.x;
  const int64_t lo = (int64_t)j * a.chunk_bytes;
  const int64_t hi = min(lo + a.chunk_bytes, a.slot_bytes);
  if (tid == 0) atomicMin((unsigned long long*)&a.result[2], (unsigned long long)now_ticks());
  for (int64_t s = 0; s < a.n_slots; ++s) {
    const int d = (int)(s % a.depth);
    const uint32_t lap = (uint32_t)(s / a.depth);
    if (tid == 0) s_ok = wait_eq(&a.freed[(int64_t)d * nwg + j], lap, a.spin_ticks, &a.result[4]);
    __syncthreads();
    if (!s_ok) return;
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(a.ring + (int64_t)d * a.slot_bytes, (short)0, (int)a.slot_bytes, 0x00020000);
    int64_t o = lo + (int64_t)tid * 16;
    // kUnroll independent 16-byte stores per thread per step, streaming and written
    // through (nt sc1): no dirty L2 line is left behind, so thread 0's release after
    // the barrier publishes the chunk
    for (; o + (kUnroll - 1) * kStep < hi; o += kUnroll * kStep) {
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int64_t ou = o + u * kStep;
        __builtin_amdgcn_raw_buffer_store_b128(pattern4(s, (uint32_t)(ou >> 2)), rs, (int)ou, 0, kStreamThrough);
      }
    }
    for (; o < hi; o += kStep) __builtin_amdgcn_raw_buffer_store_b128(pattern4(s, (uint32_t)(o >> 2)), rs, (int)o, 0, kStreamThrough);
    // every wave's written-through stores are acknowledged (performed at the
    // device's point of coherence) before the barrier, so the doorbell needs no L2
    // write-back: a relaxed store after the barrier
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) __hip_atomic_store(&a.full[(int64_t)d * nwg + j], lap + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (tid == 0) atomicMax((unsigned long long*)&a.result[3], (unsigned long long)now_ticks());
}

extern "C" __global__ __launch_bounds__(kThreads, kMinWgPerCuResident) void camelot_handoff_consumer(HandoffArgs a) {
  __shared__ int s_ok;
  __shared__ uint64_t s_sum[kWaves], s_xor[kWaves];
  const int j = blockIdx.x, nwg = gridDim.x, tid = threadIdx.x;
  const int64_t lo = (int64_t)j * a.chunk_bytes;
  const int64_t hi = min(lo + a.chunk_bytes, a.slot_bytes);
  uint64_t sum = 0;
  uint32_t xr = 0;
  for (int64_t s = 0; s < a.n_slots; ++s) {
    const int d = (int)(s % a.depth);
    const uint32_t lap = (uint32_t)(s / a.depth);
    if (tid == 0) s_ok = wait_eq(&a.full[(int64_t)d * nwg + j], lap + 1, a.spin_ticks, &a.result[4]);
    __syncthreads();
    if (!s_ok) return;
    const u32x4* base = (const u32x4*)(a.ring + (int64_t)d * a.slot_bytes);
    int64_t o = lo + (int64_t)tid * 16;
    // kUnroll independent 16-byte loads in flight per thread
    for (; o + (kUnroll - 1) * kStep < hi; o += kUnroll * kStep) {
      u32x4 v[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) v[u] = __builtin_nontemporal_load(base + ((o + u * kStep) >> 4));
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        sum += (uint64_t)v[u].x + v[u].y + v[u].z + v[u].w;
        xr ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
      }
    }
    for (; o < hi; o += kStep) {
      const u32x4 v = __builtin_nontemporal_load(base + (o >> 4));
      sum += (uint64_t)v.x + v.y + v.z + v.w;
      xr ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    __syncthreads();
    if (tid == 0) st_release_agent(&a.freed[(int64_t)d * nwg + j], lap + 1);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    sum += __shfl_xor(sum, off, 64);
    xr ^= __shfl_xor(xr, off, 64);
  }
  if ((tid & 63) == 0) { s_sum[tid >> 6] = sum; s_xor[tid >> 6] = xr; }
  __syncthreads();
  if (tid == 0) {
    uint64_t ts = 0, tx = 0;
    for (int w = 0; w < kWaves; ++w) { ts += s_sum[w]; tx ^= s_xor[w]; }
    atomicAdd((unsigned long long*)&a.result[0], (unsigned long long)ts);
    atomicXor((unsigned long long*)&a.result[1], (unsigned long long)tx);
    atomicMax((unsigned long long*)&a.result[3], (unsigned long long)now_ticks());
  }
}

}  // namespace camelot
