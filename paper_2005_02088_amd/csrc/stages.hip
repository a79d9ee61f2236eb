// Stage kernels and the persistent stage worker.
//
// One worker kernel is launched per stage instance on its CU-masked stream with one
// compute workgroup per CU of its share plus one control workgroup, the last; every
// workgroup stays resident for the life of the pipeline. The control workgroup
// forms batches (ingest or input doorbell), writes and broadcasts each batch's
// descriptor and publishes finished batches; the compute workgroups run the
// stage, separated by grid barriers where a stage has dependent phases. Every
// wait is bounded (idle limit between batches, spin limit inside a batch), so
// every wave reaches the kernel's end.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>
#include <hip/hip_fp16.h>

#include "device_common.h"

namespace camelot {

// A stage's output rows go to a ring slot that other workgroups (the next stage, on
// other XCDs) read once the batch is counted done. They are written through to the
// device's point of coherence (relaxed agent-scope atomic stores: cache policy sc1),
// so no dirty L2 line is left behind and the one release of the done count publishes
// them; with plain stores a write-back in every wave was needed, which cost the MLP
// instance ~40 us per batch when co-located.
__device__ __forceinline__ void out_f32(float* p, float v) {
  __hip_atomic_store(reinterpret_cast<uint32_t*>(p), __float_as_uint(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void out_u32(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}


typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// LOGMEL table layout (floats), built by the host (logmel_tables in runtime.cpp)
constexpr int kTabWin = 0;          // 400 Hamming window values
constexpr int kTabTw256 = 400;      // 256 complex exp(-2 pi i t / 256)
constexpr int kTabTw512 = 912;      // 257 complex exp(-2 pi i k / 512)
constexpr int kTabMelMeta = 1426;   // 40 x (first bin, bin count, weight offset)
constexpr int kTabMelW = 1546;      // concatenated filter weights

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// ------------------------------------------------------------------ result emit
// Writes one result row (k indices + k values held in LDS) either into the
// planar bench output or into the pinned egress ring. Called by a whole wave.
__device__ __forceinline__ void emit_row(const WorkerArgs& a, const BatchDesc* bd, int rows, int r,
                                         int k, const int32_t* idx, const float* val, int lane) {
  if (a.out_kind == kOutBench) {
    int32_t* ip = (int32_t*)a.bench_out;
    float* vp = (float*)(a.bench_out + (int64_t)rows * k * 4);
    for (int j = lane; j < k; j += 64) {
      ip[(int64_t)r * k + j] = idx[j];
      vp[(int64_t)r * k + j] = val[j];
    }
    return;
  }
  uint64_t slot = (bd->egress_base + (uint64_t)r) % (uint64_t)a.egress_cap;
  uint8_t* rec = a.egress + slot * (uint64_t)a.rec_bytes;
  int32_t* ip = (int32_t*)(rec + sizeof(EgressRec));
  float* vp = (float*)(ip + k);
  for (int j = lane; j < k; j += 64) {
    ip[j] = idx[j];
    vp[j] = val[j];
  }
  if (lane < 2 * kMaxStages) {
    ((EgressRec*)rec)->t_stage[lane] = bd->t_stage[lane];
  }
  if (lane == 0) {
    EgressRec* h = (EgressRec*)rec;
    h->id = bd->row_id[r];
    h->row = bd->row_idx[r];
    h->n_out = (uint32_t)k;
    h->t_arr = bd->row_tarr[r];
    h->t_done = now_ticks();
  }
}

// Where the rows of the current batch are: contiguous in the input ring slot (stages
// after the first) or in the one-shot kernel's input, at a computed address; or, for
// the first stage, wherever each request's payload put them (the per-row table
// the control workgroup fills). Kernels read rows through this, so after the batch broadcast
// no workgroup waits on a table load before its first row load.
struct BatchRows {
  const uint8_t* base;          // row r at base + r * stride, or
  int64_t stride;
  const uint8_t* const* table;  // row r at table[r]
  const BatchDesc* bd;          // the batch's descriptor (side bytes, egress records)
  __device__ __forceinline__ const uint8_t* row(int r) const {
    return base ? base + (int64_t)r * stride : table[r];
  }
};

__device__ __forceinline__ BatchRows batch_rows(const WorkerArgs& a, const BatchDesc* bd, uint64_t seq) {
  if (a.in_kind == kInRing)
    return BatchRows{a.in_ring + (seq % (uint64_t)a.in_depth) * (uint64_t)a.in_stride + kSlotHeaderBytes,
                     a.sp.in_row_bytes, nullptr, bd};
  if (a.in_kind == kInBench) return BatchRows{a.bench_in, a.in_row_stride, nullptr, bd};
  return BatchRows{nullptr, 0, bd->rowptr, bd};
}

// Workgroups that run the stage: all of them in a one-shot launch; a persistent
// worker has one more, the last, which only controls.
__device__ __forceinline__ int xwg(const WorkerArgs&) { return (int)blockIdx.x; }
__device__ __forceinline__ int xnwg(const WorkerArgs& a) { return (int)gridDim.x - a.ctl_wg; }

// After a wave has written its result rows (r0, r0 + stride, ... below rows) to the
// egress ring: a system-scope release (waits until the wave's stores are
// acknowledged), then each record's sequence word, one lane per row.
__device__ __forceinline__ void seal_rows(const WorkerArgs& a, const BatchDesc* bd, int rows, int r0, int stride,
                                          int lane) {
  if (a.out_kind != kOutEgress || r0 >= rows) return;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
  for (int r = r0 + lane * stride; r < rows; r += 64 * stride) {
    const uint64_t pos = bd->egress_base + (uint64_t)r;
    EgressRec* h = (EgressRec*)(a.egress + (pos % (uint64_t)a.egress_cap) * (uint64_t)a.rec_bytes);
    __hip_atomic_store(&h->seq, pos + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// ------------------------------------------------------------------ GEMM + ReLU (FP32)
// Unit = (64 output columns, 8 rows) per workgroup; the 4 waves split K in
// interleaved 64-wide chunks and their partial sums are added in a fixed order,
// so every output's arithmetic is independent of the batch and of the grid. A lane
// owns one column: its weight loads are 256 contiguous bytes per wave and k.
constexpr int kGemmMaxK = 1024;

__device__ void exec_gemm_relu(const WorkerArgs& a, WorkerCtl* ctl, const BatchRows& br, int rows, uint8_t* out) {
  __shared__ float xs[8][kGemmMaxK];
  __shared__ float part[kWaves][8][64];
  const int K = a.sp.dims[0], N = a.sp.dims[1];
  const float* W = (const float*)a.sp.w[0];
  float* Y = (float*)out;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int n_cb = (N + 63) / 64, n_rb = (rows + 7) / 8;
  for (int u = xwg(a); u < n_cb * n_rb; u += xnwg(a)) {
    const int cb = u % n_cb, rb = u / n_cb;
    for (int i = tid; i < 8 * K; i += kThreads) {
      const int r = i / K, kk = i - r * K, row = rb * 8 + r;
      xs[r][kk] = row < rows ? ((const float*)br.row(row))[kk] : 0.f;
    }
    __syncthreads();
    const int col = cb * 64 + lane;
    float acc[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) acc[r] = 0.f;
    if (col < N) {
      for (int kc = w * 64; kc < K; kc += kWaves * 64) {
        const int kend = min(kc + 64, K);
        int kk = kc;
        // 16 weight loads in flight before their FMAs (the FMAs keep increasing k)
        for (; kk + 16 <= kend; kk += 16) {
          float wv[16];
#pragma unroll
          for (int q = 0; q < 16; ++q) wv[q] = W[(int64_t)(kk + q) * N + col];
#pragma unroll
          for (int q = 0; q < 16; ++q)
#pragma unroll
            for (int r = 0; r < 8; ++r) acc[r] = fmaf(xs[r][kk + q], wv[q], acc[r]);
        }
        for (; kk < kend; ++kk) {
          const float wv = W[(int64_t)kk * N + col];
#pragma unroll
          for (int r = 0; r < 8; ++r) acc[r] = fmaf(xs[r][kk], wv, acc[r]);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) part[w][r][lane] = acc[r];
    __syncthreads();
    for (int i = tid; i < 8 * 64; i += kThreads) {
      const int r = i >> 6, c = i & 63, row = rb * 8 + r, cc = cb * 64 + c;
      if (row < rows && cc < N) {
        const float s = ((part[0][r][c] + part[1][r][c]) + part[2][r][c]) + part[3][r][c];
        out_f32(&Y[(int64_t)row * N + cc], fmaxf(s, 0.f));
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ GEMM + argmax (FP32)
// One wave per row: lanes stride over K, butterfly sums (lane 0's order is fixed),
// lane 0 picks the first maximum.
constexpr int kArgmaxMaxN = 16;

__device__ void exec_gemm_argmax(const WorkerArgs& a, WorkerCtl* ctl, const BatchRows& br, int rows) {
  __shared__ int32_t s_idx[kWaves][1];
  __shared__ float s_val[kWaves][1];
  const int K = a.sp.dims[0], N = a.sp.dims[1];
  const float* W = (const float*)a.sp.w[0];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int r = xwg(a) * kWaves + w; r < rows; r += xnwg(a) * kWaves) {
    const float* x = (const float*)br.row(r);
    float acc[kArgmaxMaxN];
#pragma unroll
    for (int j = 0; j < kArgmaxMaxN; ++j) acc[j] = 0.f;
    for (int kk = lane; kk < K; kk += 64) {
      const float xv = x[kk];
#pragma unroll
      for (int j = 0; j < kArgmaxMaxN; ++j)
        if (j < N) acc[j] = fmaf(xv, W[(int64_t)kk * N + j], acc[j]);
    }
#pragma unroll
    for (int j = 0; j < kArgmaxMaxN; ++j) {
      float v = acc[j];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      acc[j] = v;
    }
    if (lane == 0) {
      int best = 0;
      float bv = acc[0];
#pragma unroll
      for (int j = 1; j < kArgmaxMaxN; ++j)
        if (j < N && acc[j] > bv) { bv = acc[j]; best = j; }
      s_idx[w][0] = best;
      s_val[w][0] = bv;
    }
    wave_lds_sync();
    emit_row(a, br.bd, rows, r, 1, s_idx[w], s_val[w], lane);
    wave_lds_sync();
  }
  seal_rows(a, br.bd, rows, xwg(a) * kWaves + w, xnwg(a) * kWaves, lane);
}

// Raw buffer loads: a 32-bit per-lane offset (a scalar offset for the rest), and an
// offset past the buffer's size reads zeros, so a load needs neither a 64-bit
// address register nor clamping.
typedef int i32x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t mlp_rsrc(const void* base, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ uint4 bld16(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  const i32x4_t v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0);
  uint4 q;
  __builtin_memcpy(&q, &v, 16);
  return q;
}
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
// 16 bytes of a stage's output at byte offset off of its (wave-uniform) output
// base, written through like out_f32.
__device__ __forceinline__ void out_u32x4(uint8_t* base, uint32_t off, u32x4_t v) {
  const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(base, (short)0, 0x7fffffff, 0x00020000);
  i32x4_t q;
  __builtin_memcpy(&q, &v, 16);
  __builtin_amdgcn_raw_buffer_store_b128(q, r, (int)off, 0, 16);
}

// Stores written through to the point of coherence of the whole device (cache
// policy sc1): data another XCD reads after a grid barrier leaves no dirty L2 line
// behind, so the barrier's one release per workgroup publishes it.
constexpr int kWriteThrough = 16;      // sc1
__device__ __forceinline__ void wt_store16(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint4 v) {
  i32x4_t q;
  __builtin_memcpy(&q, &v, 16);
  __builtin_amdgcn_raw_buffer_store_b128(q, r, (int)voff, 0, kWriteThrough);
}
__device__ __forceinline__ void wt_store2(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint16_t v) {
  __builtin_amdgcn_raw_buffer_store_b16(v, r, (int)voff, 0, kWriteThrough);
}
__device__ __forceinline__ float4 u4_as_f4(uint4 u) {
  float4 f;
  __builtin_memcpy(&f, &u, 16);
  return f;
}

__device__ __forceinline__ float bld4f(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}

// ------------------------------------------------------------------ top-k
// One wave per row; the row sits in registers (lane: elements 4 (lane + 64 t) + e),
// loaded in one round. Order: larger value first, ties to the smaller index.
//
// Candidate filter: the k-th largest of the 64 lane maxima is a lower bound tau of
// the row's k-th largest value (those k maxima are k distinct elements), so every
// top-k element is >= tau. The elements >= tau (at least k) are compacted into LDS
// and each one's rank among them is counted directly; ranks below k are the
// result. When k > 64, or when more than kTopkCand elements pass the filter (heavy
// ties), k rounds of a wave-wide arg-max give the same result.
constexpr int kTopkMaxN = 4096;
constexpr int kTopkCand = 256;

__device__ __forceinline__ bool topk_better(float v1, int i1, float v2, int i2) {
  if (i2 < 0) return i1 >= 0;
  if (i1 < 0) return false;
  return v1 > v2 || (v1 == v2 && i1 < i2);
}

// k rounds of a wave-wide arg-max over the lane slices (values re-read from the
// row, which stays in cache; removed elements are tracked per lane in a bit mask).
__device__ __forceinline__ void topk_rounds(const float* s, int N, int k, int lane, int32_t* out_idx,
                                            float* out_val) {
  uint64_t removed = 0;
  for (int j = 0; j < k; ++j) {
    float bv = 0.f;
    int bi = -1;
    for (int t = 0; t < kTopkMaxN / 64; ++t) {
      const int i = lane + 64 * t;
      if (i >= N) break;
      const float v = s[i];
      if (!((removed >> t) & 1ull) && (bi < 0 || v > bv)) { bv = v; bi = i; }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const float ov = __shfl_xor(bv, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (topk_better(ov, oi, bv, bi)) { bv = ov; bi = oi; }
    }
    if (bi >= 0 && (bi & 63) == lane) removed |= 1ull << (bi >> 6);
    if (lane == 0) { out_idx[j] = bi; out_val[j] = bv; }
  }
}

__device__ void exec_topk(const WorkerArgs& a, WorkerCtl* ctl, const BatchRows& br, int rows) {
  __shared__ int32_t s_idx[kWaves][CAMELOT_MAX_K];
  __shared__ float s_val[kWaves][CAMELOT_MAX_K];
  __shared__ float c_val[kWaves][kTopkCand];
  __shared__ int32_t c_idx[kWaves][kTopkCand];
  __shared__ float m_val[kWaves][64];
  __shared__ float s_tau[kWaves];
  const int N = a.sp.dims[0], k = a.sp.k;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int ncol = (N + 255) >> 8;             // columns of 256 elements (the last may be partial)
  const bool filter = k <= 64 && min(N, 64) >= k;
  for (int r = xwg(a) * kWaves + w; r < rows; r += xnwg(a) * kWaves) {
    // the row pointer is the wave's (scalar registers: the buffer resource below is
    // then scalar too)
    const uint64_t sp = (uint64_t)br.row(r);
    const float* s = (const float*)(((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(sp >> 32)) << 32) |
                                    (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)sp));
    // the row in registers: v[4 t + e] holds element 4 (lane + 64 t) + e, 16 loads of
    // 16 bytes per lane issued together. Past N the value is -inf with an index >= N,
    // which every real element beats (larger, or equal with a smaller index), so
    // such padding never enters the result; a lane's elements are a disjoint subset,
    // so the lane maxima bound still holds.
    const __amdgpu_buffer_rsrc_t rs = mlp_rsrc(s, (int64_t)N * 4);
    uint4 raw[kTopkMaxN / 256];
#pragma unroll
    for (int t = 0; t < kTopkMaxN / 256; ++t) raw[t] = bld16(rs, (uint32_t)lane * 16u, (uint32_t)t * 1024u);
    // all 16 loads in flight before the first use (the scheduler would otherwise
    // reuse one register set and wait for each load in turn)
    __builtin_amdgcn_sched_barrier(0);
    float v[kTopkMaxN / 64];
#pragma unroll
    for (int t = 0; t < kTopkMaxN / 256; ++t) {
      const float4 q = u4_as_f4(raw[t]);
      const int i0 = 4 * (lane + 64 * t);
      v[4 * t + 0] = i0 + 0 < N ? q.x : -__builtin_inff();
      v[4 * t + 1] = i0 + 1 < N ? q.y : -__builtin_inff();
      v[4 * t + 2] = i0 + 2 < N ? q.z : -__builtin_inff();
      v[4 * t + 3] = i0 + 3 < N ? q.w : -__builtin_inff();
    }
    // threshold tau (all elements are candidates without the filter)
    float tau = -__builtin_inff();
    if (filter) {
      float m = -__builtin_inff();
#pragma unroll
      for (int j = 0; j < kTopkMaxN / 64; ++j) m = v[j] > m ? v[j] : m;
      m_val[w][lane] = m;
      wave_lds_sync();
      int rank = 0;
#pragma unroll 16
      for (int j = 0; j < 64; ++j) {
        const float o = m_val[w][j];
        rank += (o > m || (o == m && j < lane)) ? 1 : 0;
      }
      if (rank == k - 1) s_tau[w] = m;
      wave_lds_sync();
      tau = s_tau[w];
    }
    // elements of the row's columns of 256 that pass the filter
    int cnt = 0;
#pragma unroll
    for (int j = 0; j < kTopkMaxN / 64; ++j) cnt += ((j >> 2) < ncol && v[j] >= tau) ? 1 : 0;
    int incl = cnt;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int y = __shfl_up(incl, d, 64);
      if (lane >= d) incl += y;
    }
    const int C = __shfl(incl, 63, 64);
    if (C <= kTopkCand) {
      int pos = incl - cnt;
#pragma unroll
      for (int j = 0; j < kTopkMaxN / 64; ++j) {
        if ((j >> 2) < ncol && v[j] >= tau) {
          c_val[w][pos] = v[j];
          c_idx[w][pos] = 4 * (lane + 64 * (j >> 2)) + (j & 3);
          ++pos;
        }
      }
      wave_lds_sync();
      for (int c = lane; c < C; c += 64) {
        const float vc = c_val[w][c];
        const int ic = c_idx[w][c];
        int rank = 0;
#pragma unroll 8
        for (int j = 0; j < C; ++j) {
          const float o = c_val[w][j];
          rank += (o > vc || (o == vc && c_idx[w][j] < ic)) ? 1 : 0;
        }
        if (rank < k) { s_idx[w][rank] = ic; s_val[w][rank] = vc; }
      }
    } else {
      topk_rounds(s, N, k, lane, s_idx[w], s_val[w]);
    }
    wave_lds_sync();
    emit_row(a, br.bd, rows, r, k, s_idx[w], s_val[w], lane);
    wave_lds_sync();
  }
  seal_rows(a, br.bd, rows, xwg(a) * kWaves + w, xnwg(a) * kWaves, lane);
}

// ------------------------------------------------------------------ log-mel front end
// One wave per (row, frame): window 400 samples, pack into 256 complex points,
// radix-4 Stockham FFT in LDS (4 passes), split into the 257-bin spectrum of the
// 512-point real transform, power, sparse mel filters, natural log with floor.
// Each wave runs two (row, frame) units in lockstep (the LDS round trips of one hide
// behind the other's arithmetic) and loads the next pair's samples while the
// current pair is transformed.
constexpr int kTabFloats = 2304;     // room for the window, twiddles and filters

__device__ void exec_logmel(const WorkerArgs& a, WorkerCtl* ctl, const BatchRows& br, int rows, uint8_t* out) {
  // no multiply-add contraction: the two units of a pair are separate code, and a
  // frame must get the same bits in either slot (explicit fmaf calls stay fused)
#pragma clang fp contract(off)
  __shared__ float2 fbuf[kWaves][2][2][256];   // [wave][unit of the pair][ping-pong][point]
  __shared__ float pbuf[kWaves][2][260];
  __shared__ float tab[kTabFloats];
  // stage the small tables in LDS once per batch
  for (int i = threadIdx.x; i < kTabFloats; i += kThreads) tab[i] = a.sp.tables[i];
  __syncthreads();
  const float* win = tab + kTabWin;
  const float2* tw256 = (const float2*)(tab + kTabTw256);
  const float2* tw512 = (const float2*)(tab + kTabTw512);
  const float* meta = tab + kTabMelMeta;
  const float* melw = tab + kTabMelW;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  float* Y = (float*)out;
  const int units = rows * 11, stride = xnwg(a) * kWaves;
  // the samples of a (row, frame) unit: 200 float2 per frame, lane + 64 q (global
  // loads, no branches: the last piece is clamped)
  typedef float f32x2_t __attribute__((ext_vector_type(2)));
  typedef const f32x2_t __attribute__((address_space(1)))* gptr_f2;
  f32x2_t xr[2][4];
  auto load_unit = [&](int slot, int uu) {
    const int r = uu / 11, f = uu - r * 11;
    const gptr_f2 x2 = (gptr_f2)((const float*)br.row(r) + f * 160);
#pragma unroll
    for (int q = 0; q < 3; ++q) xr[slot][q] = x2[lane + 64 * q];
    xr[slot][3] = x2[lane + 192 < 200 ? lane + 192 : 199];
  };
  // pairs (u, u + stride); a pair without a second unit runs its first twice and
  // stores once
  int u = xwg(a) * kWaves + w;
  if (u < units) {
    load_unit(0, u);
    load_unit(1, u + stride < units ? u + stride : u);
  }
  for (; u < units; u += 2 * stride) {
    const int u1 = u + stride < units ? u + stride : u;
    const bool second = u + stride < units;
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int n = lane + 64 * q;
        float2 z = make_float2(0.f, 0.f);
        if (n < 200) z = make_float2(xr[sl][q].x * win[2 * n], xr[sl][q].y * win[2 * n + 1]);
        fbuf[w][sl][0][n] = z;
      }
    }
    {
      const int un = u + 2 * stride;
      if (un < units) {
        load_unit(0, un);
        load_unit(1, un + stride < units ? un + stride : un);
      }
    }
    wave_lds_sync();
    int src = 0;
    for (int ns = 1; ns < 256; ns *= 4) {
      const int j = lane, jm = j % ns, step = 64 / ns;
      const int d = (j / ns) * ns * 4 + jm;
      float2 y[2][4];
#pragma unroll
      for (int sl = 0; sl < 2; ++sl) {
        float2 v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float2 e = fbuf[w][sl][src][j + 64 * q];
          const float2 t = tw256[q * jm * step];
          v[q] = make_float2(e.x * t.x - e.y * t.y, e.x * t.y + e.y * t.x);
        }
        // forward radix-4 butterfly (omega = -i)
        const float2 s02 = make_float2(v[0].x + v[2].x, v[0].y + v[2].y);
        const float2 d02 = make_float2(v[0].x - v[2].x, v[0].y - v[2].y);
        const float2 s13 = make_float2(v[1].x + v[3].x, v[1].y + v[3].y);
        const float2 d13 = make_float2(v[1].x - v[3].x, v[1].y - v[3].y);
        y[sl][0] = make_float2(s02.x + s13.x, s02.y + s13.y);
        y[sl][2] = make_float2(s02.x - s13.x, s02.y - s13.y);
        y[sl][1] = make_float2(d02.x + d13.y, d02.y - d13.x);   // d02 - i d13
        y[sl][3] = make_float2(d02.x - d13.y, d02.y + d13.x);   // d02 + i d13
      }
#pragma unroll
      for (int sl = 0; sl < 2; ++sl)
#pragma unroll
        for (int q = 0; q < 4; ++q) fbuf[w][sl][src ^ 1][d + q * ns] = y[sl][q];
      wave_lds_sync();
      src ^= 1;
    }
    for (int kk = lane; kk <= 256; kk += 64) {
      const float2 t = tw512[kk];
#pragma unroll
      for (int sl = 0; sl < 2; ++sl) {
        const float2 za = fbuf[w][sl][src][kk & 255];
        const float2 zb = fbuf[w][sl][src][(256 - kk) & 255];
        const float er = 0.5f * (za.x + zb.x), ei = 0.5f * (za.y - zb.y);
        const float dr = za.x - zb.x, di = za.y + zb.y;            // a - conj(b)
        const float orr = 0.5f * di, oi = -0.5f * dr;               // (a - conj b) / 2i
        const float xr_ = er + (t.x * orr - t.y * oi);
        const float xi_ = ei + (t.x * oi + t.y * orr);
        pbuf[w][sl][kk] = xr_ * xr_ + xi_ * xi_;
      }
    }
    wave_lds_sync();
    if (lane < 40) {
      const int lo = (int)meta[3 * lane], cnt = (int)meta[3 * lane + 1], off = (int)meta[3 * lane + 2];
      float e0 = 0.f, e1 = 0.f;
#pragma unroll 4
      for (int t = 0; t < cnt; ++t) {
        const float wt = melw[off + t];
        e0 = fmaf(wt, pbuf[w][0][lo + t], e0);
        e1 = fmaf(wt, pbuf[w][1][lo + t], e1);
      }
      const int r0 = u / 11, f0 = u - r0 * 11;
      out_f32(&Y[(int64_t)r0 * 440 + f0 * 40 + lane], logf(fmaxf(e0, 1e-10f)));
      if (second) {
        const int r1 = u1 / 11, f1 = u1 - r1 * 11;
        out_f32(&Y[(int64_t)r1 * 440 + f1 * 40 + lane], logf(fmaxf(e1, 1e-10f)));
      }
    }
    wave_lds_sync();
  }
}

// ------------------------------------------------------------------ BF16 MLP chain on MFMA
// 16-byte load from global memory (explicitly in the global address space, so it
// is a global load counted by vmcnt only, never a flat load that also holds up
// every LDS wait).
typedef const u32x4_t __attribute__((address_space(1)))* gptr_u32x4;
__device__ __forceinline__ uint4 gld16(const void* p) {
  const u32x4_t v = *(gptr_u32x4)p;
  uint4 r;
  __builtin_memcpy(&r, &v, 16);
  return r;
}

__device__ __forceinline__ bf16x8 ld_bf16x8(const uint16_t* p) {
  const uint4 q = gld16(p);
  bf16x8 r;
  __builtin_memcpy(&r, &q, 16);
  return r;
}

__device__ __forceinline__ uint4 f32x8_to_bf16x8_bits(const float4 a, const float4 b) {
  uint4 q;
  q.x = (uint32_t)f32_to_bf16_rne(a.x) | ((uint32_t)f32_to_bf16_rne(a.y) << 16);
  q.y = (uint32_t)f32_to_bf16_rne(a.z) | ((uint32_t)f32_to_bf16_rne(a.w) << 16);
  q.z = (uint32_t)f32_to_bf16_rne(b.x) | ((uint32_t)f32_to_bf16_rne(b.y) << 16);
  q.w = (uint32_t)f32_to_bf16_rne(b.z) | ((uint32_t)f32_to_bf16_rne(b.w) << 16);
  return q;
}

// Per layer, out = act W^T with W [N][K] BF16 (K contiguous), on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation; ReLU and BF16 rounding for the
// hidden layers, an FP32 store for the last; layers are separated by grid barriers.
// A unit is (up to 4 RW row blocks of 16 rows) x (CT column strips of 16); wave w
// owns row blocks w, w + 4, ... of the unit and runs the whole K for them, one MFMA
// chain per output tile in increasing K order. Every output element's sum therefore
// has one fixed order, whatever the batch, the row's position, the unit shape or
// the grid, and a row's result does not depend on the other rows.
//
// K is walked in stages of 4 chunks of 32. The stage's B (the weights, the same for
// all 4 waves) is loaded once per workgroup, spread over its 256 threads with
// row-contiguous 16-byte loads (16 lanes cover one weight row's 256 bytes), into a
// double-buffered LDS stage that the waves read as MFMA fragments (an MFMA fragment
// loaded from global memory directly would touch 4 cache lines per group of 4
// lanes). The hidden state between layers is stored in MFMA fragment order, so the
// A fragments of the next layer are single contiguous 1 KiB loads straight into
// registers; the first layer's FP32 rows are loaded row-contiguously and go
// through a per-wave LDS region. Load group g = (A of stage g, B of stage g + 1)
// sits in register slot g mod PA, PA groups in flight. Per stage: B of the next
// stage (and for FP32 rows A of this stage) go from registers to LDS, the MFMAs run,
// group g + PA is issued into the freed slot, one workgroup barrier.
constexpr int kRowPitch = 256 + 16;    // one row's stage in LDS, padded (rows on other banks)

template <int RW, int CT, bool F32>
struct MlpRowSlot {
  uint4 a[4 * RW][F32 ? 2 : 1];  // A pieces (BF16 x 8, or FP32 x 8 rounded when stored to LDS)
  uint4 b[CT];                   // this thread's pieces of the next stage's B
};

// Where this thread's loads of a unit start (stage 0). A piece m of lane L is
// segment L % 16 (8 elements) of wave row rho = 4 m + L / 16, i.e. row block
// w + 4 (rho / 16), row rho % 16 of it. BF16 rows past the batch read whatever the
// hidden state holds there (only their own, never stored, outputs see it); FP32
// rows past the batch read row 0. B piece q of thread tid is segment p % 16 of
// strip row p / 16, p = tid + 256 q.
template <int RW, int CT, bool F32>
struct MlpRowSrc {
  const float* arow[F32 ? 4 * RW : 1];
  uint32_t aoff[F32 ? 1 : RW];
  uint32_t boff[CT];
  __amdgpu_buffer_rsrc_t ra, rb;
};

template <int RW, int CT, bool F32>
__device__ __forceinline__ void mlp_row_sources(MlpRowSrc<RW, CT, F32>& src, const BatchRows& br,
                                                const uint16_t* hin, int stride, const uint16_t* W, int K, int N,
                                                int rows, int row0, int col0, int w, int lane, int tid) {
  if constexpr (F32) {
#pragma unroll
    for (int m = 0; m < 4 * RW; ++m) {
      const int rho = 4 * m + (lane >> 4);
      const int r = row0 + (w + 4 * (rho >> 4)) * 16 + (rho & 15);
      src.arow[m] = (const float*)br.row(r < rows ? r : 0) + (lane & 15) * 8;
    }
  } else {
    // the hidden state is in fragment order: row block rb, chunk c at
    // (rb nck + c) KiB, lane l's 16 bytes at 16 l (rows past the batch hold
    // whatever is there; only their own, never stored, outputs see it)
    const int nck = (K + 31) >> 5;
#pragma unroll
    for (int j = 0; j < RW; ++j) src.aoff[j] = (uint32_t)((((row0 >> 4) + w + 4 * j) * nck * 64 + lane) * 16);
  }
#pragma unroll
  for (int q = 0; q < CT; ++q) {
    const int p = tid + kThreads * q;
    src.boff[q] = (uint32_t)(((col0 + (p >> 4)) * K + (p & 15) * 8) * 2);
  }
  src.ra = mlp_rsrc(hin, (int64_t)kMaxBatch * stride * 2);
  src.rb = mlp_rsrc(W, (int64_t)N * K * 2);
}

// B pieces of stage st (past K within a row: the next row's weights, zeroed at
// use; past the matrix: zeros).
template <int RW, int CT, bool F32>
__device__ __forceinline__ void mlp_row_issue_b(uint4 (&b)[CT], const MlpRowSrc<RW, CT, F32>& src, int st) {
#pragma unroll
  for (int q = 0; q < CT; ++q) b[q] = bld16(src.rb, src.boff[q], (uint32_t)st * 256u);
}

// Load group st (A of stage st, B of stage st + 1). Stages past the last one with
// data (stl) re-load stage stl (the pipeline runs ahead of the end; those values
// are never used), so the over-run costs cache hits, not memory traffic.
template <int RW, int CT, bool F32>
__device__ __forceinline__ void mlp_row_issue(MlpRowSlot<RW, CT, F32>& r, const MlpRowSrc<RW, CT, F32>& src, int K,
                                              int st, int stl, int lane) {
  const int sa = min(st, stl);
#pragma unroll
  for (int m = 0; m < 4 * RW; ++m) {
    if constexpr (F32) {
      // FP32 rows come from separate buffers: clamped global loads (K past the end
      // reads column 0; zeroed at use)
      const int k = sa * 128 + (lane & 15) * 8;
      const float* p = src.arow[m] + (k < K ? sa * 128 : -(lane & 15) * 8);
      r.a[m][0] = gld16(p);
      r.a[m][1] = gld16(p + 4);
    } else {
      // fragment m = c RW + j: chunk c of the stage, row block j
      r.a[m][0] = bld16(src.ra, src.aoff[m % RW] + (m / RW) * 1024u, (uint32_t)sa * 4096u);
    }
  }
  mlp_row_issue_b<RW, CT, F32>(r.b, src, min(st + 1, stl));
}

template <int CT>
__device__ __forceinline__ void mlp_row_stash_b(const uint4 (&b)[CT], uint8_t* buf, int tid) {
#pragma unroll
  for (int q = 0; q < CT; ++q) {
    const int p = tid + kThreads * q;
    *(uint4*)(buf + (p >> 4) * kRowPitch + (p & 15) * 16) = b[q];
  }
}

// This wave's A pieces of the stage into its LDS region (FP32 rounded to BF16).
template <int RW, int CT, bool F32>
__device__ __forceinline__ void mlp_row_stash_a(const MlpRowSlot<RW, CT, F32>& r, uint8_t* reg, int lane) {
#pragma unroll
  for (int m = 0; m < 4 * RW; ++m) {
    const int rho = 4 * m + (lane >> 4);
    uint4 v;
    if constexpr (F32) v = f32x8_to_bf16x8_bits(u4_as_f4(r.a[m][0]), u4_as_f4(r.a[m][1]));
    else v = r.a[m][0];
    *(uint4*)(reg + rho * kRowPitch + (lane & 15) * 16) = v;
  }
}

// Fragments of chunk c of a stage: B from LDS; A from the wave's LDS region (FP32
// rows, staged) or straight from the slot registers (the hidden state, loaded in
// fragment order). TAIL zeroes A and B past K.
template <int RW, int CT>
struct MlpRowFrag {
  bf16x8 a[RW], b[CT];
};

template <int RW, int CT, bool F32, bool TAIL>
__device__ __forceinline__ void mlp_row_frag(MlpRowFrag<RW, CT>& f, const MlpRowSlot<RW, CT, F32>& sl,
                                             const uint8_t* areg, const uint8_t* buf, int fo, int c, bool tail) {
#pragma unroll
  for (int j = 0; j < RW; ++j) {
    if constexpr (F32) {
      f.a[j] = *(const bf16x8*)(areg + j * 16 * kRowPitch + fo + c * 64);
      if (TAIL && tail) f.a[j] = (bf16x8){};
    } else if constexpr (TAIL) {
      __builtin_memcpy(&f.a[j], &sl.a[c * RW + j][0], 16);
      if (tail) f.a[j] = (bf16x8){};
    }
  }
#pragma unroll
  for (int t = 0; t < CT; ++t) {
    f.b[t] = *(const bf16x8*)(buf + t * 16 * kRowPitch + fo + c * 64);
    if (TAIL && tail) f.b[t] = (bf16x8){};
  }
}

// A operand: the fragment read into f (FP32 rows, or a zeroed tail), else the slot
// register itself (no copy).
template <int RW, int CT, bool F32, bool TAIL>
__device__ __forceinline__ void mlp_row_mfma_chunk(f32x4 (&acc)[RW][CT], const MlpRowFrag<RW, CT>& f,
                                                   const MlpRowSlot<RW, CT, F32>& sl, int c) {
#pragma unroll
  for (int t = 0; t < CT; ++t)
#pragma unroll
    for (int j = 0; j < RW; ++j) {
      bf16x8 av;
      if constexpr (F32 || TAIL) av = f.a[j];
      else __builtin_memcpy(&av, &sl.a[c * RW + j][0], 16);
      acc[j][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, f.b[t], acc[j][t], 0, 0, 0);
    }
}

// MFMAs of one stage. A stage inside K is straight-line code with the fragments of
// chunk c + 1 read while the MFMAs of chunk c run; the last stage skips the chunks
// past K and zeroes the K tail.
template <int RW, int CT, bool F32>
__device__ __forceinline__ void mlp_row_mfma(f32x4 (&acc)[RW][CT], const MlpRowSlot<RW, CT, F32>& sl,
                                             const uint8_t* areg, const uint8_t* buf, int K, int st, int lane) {
  const int fo = (lane & 15) * kRowPitch + (lane >> 4) * 16;
  if ((st + 1) * 128 <= K) {
    MlpRowFrag<RW, CT> f[2];
    mlp_row_frag<RW, CT, F32, false>(f[0], sl, areg, buf, fo, 0, false);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      if (c < 3) mlp_row_frag<RW, CT, F32, false>(f[(c + 1) & 1], sl, areg, buf, fo, c + 1, false);
      __builtin_amdgcn_sched_barrier(0);
      mlp_row_mfma_chunk<RW, CT, F32, false>(acc, f[c & 1], sl, c);
      __builtin_amdgcn_sched_barrier(0);
    }
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int k0 = st * 128 + c * 32;
      if (k0 < K) {
        MlpRowFrag<RW, CT> f;
        mlp_row_frag<RW, CT, F32, true>(f, sl, areg, buf, fo, c, k0 + 32 > K && k0 + (lane >> 4) * 8 >= K);
        mlp_row_mfma_chunk<RW, CT, F32, true>(acc, f, sl, c);
      }
    }
  }
}

// Load groups in flight per unit shape. All shapes are compiled into one kernel, whose
// registers are those of its hungriest path, so the depths are chosen together: as
// deep as the whole kernel stays within 256 registers per lane with no spills. A
// worker kernel must not need scratch (the launch refuses one that does): the
// runtime may start fewer waves of a kernel than its grid when it cannot back the
// scratch of all of them at once, and a persistent grid whose workgroups are not all
// resident never completes a grid barrier. (Eight groups for the narrow BF16 units
// would spill.) At least two: the B stage of the next group is written while the
// MFMAs read the current one, so there are always two B buffers.
#ifndef MLP_PA
#define MLP_PA(RW, CT, F32) ((F32) ? ((RW) == 2 ? 2 : 4) : (RW) == 2 ? 2 : 4)
#endif
// LDS of the row path: the waves' A regions (FP32 rows), then the B stage buffers
constexpr int kMlpRowLds = 8 * 32 * kRowPitch;

// One unit: rows row0 .. row0 + 64 RW - 1 (wave w: row blocks w, w + 4, ...),
// columns col0 .. col0 + 16 CT - 1. All 4 waves run every stage (the barriers).
template <int RW, int CT, bool F32>
__device__ __forceinline__ void mlp_row_unit(const BatchRows& br, const uint16_t* hin, int stride,
                                             const uint16_t* W, int K, int N, int rows, int row0, int col0,
                                             bool last, uint16_t* hout, float* out, uint8_t* lds, int w, int lane,
                                             int tid) {
  constexpr int PA = MLP_PA(RW, CT, F32);                       // load groups in flight
  constexpr int NB = (PA % 2 == 0) ? 2 : PA;                    // B stage buffers
  static_assert(PA >= 2 && PA % NB == 0, "two B buffers at least; buffer of a stage known at compile time");
  constexpr int SB = 16 * CT * kRowPitch;                       // bytes of one B stage buffer
  constexpr int SA = F32 ? 16 * RW * kRowPitch : 0;             // a wave's A region (FP32 rows only)
  static_assert(4 * SA + NB * SB <= kMlpRowLds, "row path LDS");
  uint8_t* areg = lds + w * SA;
  uint8_t* bbuf = lds + 4 * SA;
  MlpRowSrc<RW, CT, F32> src;
  mlp_row_sources<RW, CT, F32>(src, br, hin, stride, W, K, N, rows, row0, col0, w, lane, tid);
  f32x4 acc[RW][CT];
#pragma unroll
  for (int j = 0; j < RW; ++j)
#pragma unroll
    for (int t = 0; t < CT; ++t) acc[j][t] = (f32x4){0.f, 0.f, 0.f, 0.f};
  // stages padded to a multiple of PA (padding stages load and do no MFMAs)
  const int ns = ((K + 127) / 128 + PA - 1) / PA * PA;
  const int stl = (K + 127) / 128 - 1;      // the last stage with data
  MlpRowSlot<RW, CT, F32> sl[PA];
  {
    uint4 b0[CT];
    __builtin_amdgcn_sched_barrier(0);
    mlp_row_issue_b<RW, CT, F32>(b0, src, 0);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int g = 0; g < PA; ++g) {
      mlp_row_issue<RW, CT, F32>(sl[g], src, K, g, stl, lane);
      __builtin_amdgcn_sched_barrier(0);
    }
    mlp_row_stash_b<CT>(b0, bbuf, tid);
    __syncthreads();
  }
  for (int s = 0; s < ns; s += PA) {
#pragma unroll
    for (int i = 0; i < PA; ++i) {
      const int st = s + i;                 // s is a multiple of NB: the buffer of stage st is i % NB
      __builtin_amdgcn_sched_barrier(0);
      mlp_row_stash_b<CT>(sl[i].b, bbuf + ((i + 1) % NB) * SB, tid);
      if constexpr (F32) {
        mlp_row_stash_a<RW, CT, F32>(sl[i], areg, lane);
        // the wave's own A region: its writes are in place before its reads
        wave_lds_sync();
      }
      __builtin_amdgcn_sched_barrier(0);
      mlp_row_mfma<RW, CT, F32>(acc, sl[i], areg, bbuf + (i % NB) * SB, K, st, lane);
      __builtin_amdgcn_sched_barrier(0);
      mlp_row_issue<RW, CT, F32>(sl[i], src, K, st + PA, stl, lane);
      __builtin_amdgcn_sched_barrier(0);
      __syncthreads();
    }
  }
  const int nckn = (N + 31) >> 5;
  const __amdgpu_buffer_rsrc_t rh = mlp_rsrc(hout, (int64_t)kMaxBatch * nckn * 32 * 2);
#pragma unroll
  for (int j = 0; j < RW; ++j) {
#pragma unroll
    for (int t = 0; t < CT; ++t) {
      const int col = col0 + t * 16 + (lane & 15);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = row0 + (w + 4 * j) * 16 + (lane >> 4) * 4 + i;
        if (row < rows) {
          const float v = acc[j][t][i];
          if (last) {
            out_f32(&out[(int64_t)row * N + col], v);
          } else {
            // the next layer reads the hidden state in fragment order (row block,
            // 32-wide chunk, lane = row % 16 + 16 ((col % 32) / 8), element col % 8)
            const int64_t e = ((int64_t)((row >> 4) * nckn + (col >> 5)) * 64 + (row & 15) + 16 * ((col & 31) >> 3)) * 8 +
                              (col & 7);
            wt_store2(rh, (uint32_t)(e * 2), f32_to_bf16_rne(fmaxf(v, 0.f)));
          }
        }
      }
    }
  }
}

template <int RW, int CT, bool F32>
__device__ __forceinline__ void mlp_row_layer(const BatchRows& br, const uint16_t* hin, int stride,
                                              const uint16_t* W, int K, int N, int rows, bool last, uint16_t* hout,
                                              float* out, uint8_t* lds, int w, int lane, int tid, int wgi, int nwg) {
  const int rpu = 4 * RW;                               // row blocks per unit
  const int nrg = (((rows + 15) >> 4) + rpu - 1) / rpu, ncb = N / (16 * CT);
  for (int u = wgi; u < nrg * ncb; u += nwg) {
    const int cb = u % ncb, row0 = (u / ncb) * rpu * 16;
    mlp_row_unit<RW, CT, F32>(br, hin, stride, W, K, N, rows, row0, cb * 16 * CT, last, hout, out, lds, w,
                              lane, tid);
  }
}

// The batch's FP32 input rows rounded to BF16 (nearest even, as the FP32 unit path
// rounds them) into the hidden-state buffer in fragment order, zeros past K; rows
// past the batch are not written. Threads take consecutive 8-element groups of a
// row, so the reads are contiguous.
__device__ __forceinline__ void mlp_input_to_frag(const BatchRows& br, uint16_t* h, int K, int rows, int wgi, int nwg) {
  const int nck = (K + 31) >> 5, ngr = nck * 4;             // 8-element groups per padded row
  const int total = rows * ngr;
  const __amdgpu_buffer_rsrc_t rh = mlp_rsrc(h, (int64_t)kMaxBatch * nck * 32 * 2);
  for (int i = wgi * kThreads + threadIdx.x; i < total; i += nwg * kThreads) {
    const int row = i / ngr, g = i - row * ngr, k0 = g * 8;
    uint4 v = {0u, 0u, 0u, 0u};
    if (k0 < K) {
      const float* x = (const float*)br.row(row) + k0;
      v = f32x8_to_bf16x8_bits(u4_as_f4(gld16(x)), u4_as_f4(gld16(x + 4)));
    }
    const int c = g >> 2, lane = (row & 15) + 16 * (g & 3);
    wt_store16(rh, (uint32_t)((((row >> 4) * nck + c) * 64 + lane) * 16), v);
  }
}

// One layer on the BF16 (fragment-order) input. The unit shape (row blocks x column
// strips: 8 x 4, 8 x 2, 4 x 2 or 4 x 1) is the one with the least work on the
// busiest workgroup: rounds of the grid (ceil(units / workgroups)) times a unit's
// cost, the activation and weight bytes it streams ((row blocks + strips) per K
// element) plus a fixed per-unit cost of about three stages (pipeline fill, stores).
// A shape that fits in fewer rounds wins on a larger share only if it is cheaper,
// so the layer's time never grows when CUs are added; ties go to the larger unit.
// Every shape gives the same bits (one MFMA chain per output in K order).
__device__ __forceinline__ int mlp_bf16_shape(int nrt, int N, int K, int P) {
  constexpr int kRw[4] = {2, 2, 1, 1}, kCt[4] = {4, 2, 2, 1};
  int best = 3;
  int64_t best_cost = INT64_MAX;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int rw = kRw[i], ct = kCt[i], rpu = 4 * rw;
    if (N % (16 * ct) != 0 || (rw == 2 && nrt <= 4)) continue;
    const int units = ((nrt + rpu - 1) / rpu) * (N / (16 * ct));
    const int64_t rounds = (units + P - 1) / P;
    const int64_t cost = rounds * (int64_t)(K + 3 * 128) * (rpu + ct);
    if (cost < best_cost) {
      best_cost = cost;
      best = i;
    }
  }
  return best;
}

__device__ __forceinline__ void mlp_bf16_layer(const BatchRows& rp, const uint16_t* hin, int stride, const uint16_t* W,
                                               int K, int N, int rows, bool last, uint16_t* hout, float* o,
                                               uint8_t* lds, int w, int lane, int tid, int wgi, int nwg) {
  switch (mlp_bf16_shape((rows + 15) >> 4, N, K, nwg)) {
    case 0: mlp_row_layer<2, 4, false>(rp, hin, stride, W, K, N, rows, last, hout, o, lds, w, lane, tid, wgi, nwg); break;
    case 1: mlp_row_layer<2, 2, false>(rp, hin, stride, W, K, N, rows, last, hout, o, lds, w, lane, tid, wgi, nwg); break;
    case 2: mlp_row_layer<1, 2, false>(rp, hin, stride, W, K, N, rows, last, hout, o, lds, w, lane, tid, wgi, nwg); break;
    default: mlp_row_layer<1, 1, false>(rp, hin, stride, W, K, N, rows, last, hout, o, lds, w, lane, tid, wgi, nwg); break;
  }
}

// All layers of a batch. The first layer reads the FP32 input rows: the units read
// and round them themselves (unit shapes (8 x 2), (4 x 2), (4 x 1)) when one round of
// the grid covers them, or, for batches of more than 32 rows whose units would take
// two or more rounds, the rows are first rounded into fragment order once for the
// whole grid (one more grid barrier) and the layer runs like the others. Both give
// the same bits.
__device__ __forceinline__ bool mlp_rows_all(const WorkerArgs& a, WorkerCtl* ctl, const BatchRows& rp, int rows, uint8_t* out,
                                             uint8_t* lds, int w, int lane, int tid) {
  const int L = a.sp.n_layers, stride = a.sp.scratch_stride;
  const int wgi = xwg(a), nwg = xnwg(a);
  const int nrt = (rows + 15) >> 4, P = nwg;
  for (int l = 0; l < L; ++l) {
    // the hidden state is written through: one release per workgroup publishes it
    if (l > 0 && !grid_barrier(ctl, nwg, a.spin_ticks, false, wgi, false)) return false;
    const int K = a.sp.dims[l], N = a.sp.dims[l + 1];
    uint16_t* hout = a.sp.scratch + (int64_t)(l & 1) * kMaxBatch * stride;
    uint16_t* hin = a.sp.scratch + (int64_t)((l + 1) & 1) * kMaxBatch * stride;
    const uint16_t* W = (const uint16_t*)a.sp.w[l];
    const bool last = (l == L - 1);
    float* o = (float*)out;
    if (l == 0) {
      // units of the FP32 path: rounding the rows once pays when they would be read
      // by two or more rounds of units
      const bool even = (N % 32) == 0;
      const int u22 = ((nrt + 7) / 8) * (N / 32), u12 = ((nrt + 3) / 4) * (N / 32);
      const int shape = (even && nrt > 4 && u22 >= P) ? 2 : (even && u12 >= P) ? 1 : 0;
      const int units = shape == 2 ? u22 : shape == 1 ? u12 : ((nrt + 3) / 4) * (N / 16);
      if (nrt <= 2 || units <= P) {
        if (shape == 2)
          mlp_row_layer<2, 2, true>(rp, hin, stride, W, K, N, rows, last, hout, o, lds, w, lane, tid, wgi, nwg);
        else if (shape == 1)
          mlp_row_layer<1, 2, true>(rp, hin, stride, W, K, N, rows, last, hout, o, lds, w, lane, tid, wgi, nwg);
        else
          mlp_row_layer<1, 1, true>(rp, hin, stride, W, K, N, rows, last, hout, o, lds, w, lane, tid, wgi, nwg);
        continue;
      }
      mlp_input_to_frag(rp, hin, K, rows, wgi, nwg);
      if (!grid_barrier(ctl, nwg, a.spin_ticks, false, wgi, false)) return false;
    }
    mlp_bf16_layer(rp, hin, stride, W, K, N, rows, last, hout, o, lds, w, lane, tid, wgi, nwg);
  }
  return true;
}

__device__ __forceinline__ bool exec_mlp(const WorkerArgs& a, WorkerCtl* ctl, const BatchRows& br, int rows, uint8_t* out) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[kMlpRowLds];
  // the wave index is uniform across the wave: in a scalar register the per-wave
  // conditions become scalar branches instead of exec-mask regions
  const int tid = threadIdx.x, w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  return mlp_rows_all(a, ctl, br, rows, out, lds, w, lane, tid);
}

// ------------------------------------------------------------------ embedding gather
// One wave per row: the row's ids are read once (lanes < n_ids) and broadcast; every
// lane owns dim/64 columns and adds the FP16 table rows in id order in FP32, so a
// row's result does not depend on the batch. Ids outside [0, table rows) add zero.
constexpr int kGatherMaxDim = 1024;

__device__ void exec_gather(const WorkerArgs& a, WorkerCtl* ctl, const BatchRows& br, int rows, uint8_t* out) {
  const int n_ids = a.sp.dims[0], dim = a.sp.dims[1];
  const int64_t trows = a.sp.k;
  const __half* T = (const __half*)a.sp.w[0];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int per = dim >> 6;                  // columns per lane (dim is a multiple of 64)
  float* Y = (float*)out;
  for (int r = xwg(a) * kWaves + w; r < rows; r += xnwg(a) * kWaves) {
    const int32_t* ids = (const int32_t*)br.row(r);
    float acc[kGatherMaxDim / 64];
#pragma unroll
    for (int c = 0; c < kGatherMaxDim / 64; ++c) acc[c] = 0.f;
    for (int j0 = 0; j0 < n_ids; j0 += 64) {
      const int my = j0 + lane < n_ids ? ids[j0 + lane] : -1;
      const int nj = min(64, n_ids - j0);
      for (int j = 0; j < nj; ++j) {
        const int id = __shfl(my, j, 64);
        if (id < 0 || id >= trows) continue;          // uniform across the wave
        const __half* src = T + (int64_t)id * dim;
#pragma unroll
        for (int c = 0; c < kGatherMaxDim / 64; ++c)
          if (c < per) acc[c] += __half2float(src[c * 64 + lane]);
      }
    }
    const float inv = 1.f / (float)n_ids;
#pragma unroll
    for (int c = 0; c < kGatherMaxDim / 64; ++c)
      if (c < per) out_f32(&Y[(int64_t)r * dim + c * 64 + lane], acc[c] * inv);
  }
}

// ------------------------------------------------------------------ 3x3 convolution + global pool
// Implicit GEMM on v_mfma_f32_16x16x32_bf16: per query, M = H*W output pixels,
// N = 64 output channels, K = 9 positions x 64 input channels (chunks of 32 input
// channels at one (ky, kx)). A workgroup computes a 64-pixel tile (16 per wave) for
// all 64 channels, applies ReLU and sums its pixels per channel in a fixed order
// (within a wave: rows, then the 4 lane groups; then the 4 waves); phase 2, after a
// grid barrier, adds the tiles of each query in tile order and divides by H*W.
// The weights (64 x 576 BF16, 72 KiB) are staged in LDS once per batch and the B
// fragments read from there: 16-byte granule g of output channel n sits at
// n * 72 + (g ^ ((n >> 1) & 7)), so the 16 channels a fragment read touches fall on
// 16 distinct groups of 4 banks (a row is 1,152 bytes: without the swizzle, rows two
// apart share banks). A wave's 18 A fragments of a tile (9 positions x 2 chunks) are
// loaded before its first MFMA.
constexpr int kConvC = 64, kConvCout = 64, kConvTile = 64;
constexpr int kConvRowGran = 9 * kConvC / 8;           // 16-byte granules per output channel

__device__ bool exec_conv_pool(const WorkerArgs& a, WorkerCtl* ctl, const BatchRows& br, int rows, uint8_t* out) {
  __shared__ float wsum[kWaves][kConvCout];
  __shared__ __attribute__((aligned(16))) uint4 wl[kConvCout * kConvRowGran];
  const int H = a.sp.dims[0], Wd = a.sp.dims[1];
  const int npix = H * Wd, ntiles = (npix + kConvTile - 1) / kConvTile;
  const uint16_t* Wc = (const uint16_t*)a.sp.w[0];          // [64][9][64]
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int units = rows * ntiles;
  if (xwg(a) < units) {
    for (int i = tid; i < kConvCout * kConvRowGran; i += kThreads) {
      const int n = i / kConvRowGran, g = i - n * kConvRowGran;
      wl[n * kConvRowGran + (g ^ ((n >> 1) & 7))] = gld16(Wc + (int64_t)n * (9 * kConvC) + g * 8);
    }
    __syncthreads();
  }
  const int bn = lane & 15;                                  // this lane's output channel within a block of 16
  for (int u = xwg(a); u < units; u += xnwg(a)) {
    const int r = u / ntiles, tile = u - r * ntiles;
    const uint16_t* X = (const uint16_t*)br.row(r);
    const int p = tile * kConvTile + w * 16 + (lane & 15);   // A-operand pixel of this lane
    const int py = p / Wd, px = p - py * Wd;
    const bool pin = p < npix;
    bf16x8 af[9][2];
#pragma unroll
    for (int pos = 0; pos < 9; ++pos) {
      const int ky = pos / 3, kx = pos - ky * 3;
      const int yy = py + ky - 1, xx = px + kx - 1;
      const bool in = pin && yy >= 0 && yy < H && xx >= 0 && xx < Wd;
      const uint16_t* xs = X + ((int64_t)yy * Wd + xx) * kConvC + (lane >> 4) * 8;
#pragma unroll
      for (int h = 0; h < 2; ++h) af[pos][h] = in ? ld_bf16x8(xs + h * 32) : (bf16x8){};
    }
    f32x4 acc[4];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) acc[nb] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int pos = 0; pos < 9; ++pos) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int g = pos * 8 + h * 4 + (lane >> 4);         // this lane's 8 input channels at (ky, kx)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
          const int n = nb * 16 + bn;
          bf16x8 bf;
          const uint4 q = wl[n * kConvRowGran + (g ^ ((n >> 1) & 7))];
          __builtin_memcpy(&bf, &q, 16);
          acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[pos][h], bf, acc[nb], 0, 0, 0);
        }
      }
    }
    // ReLU and the sum over this wave's 16 pixels per channel
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
      float v = 0.f;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int pr = tile * kConvTile + w * 16 + (lane >> 4) * 4 + i;
        if (pr < npix) v += fmaxf(acc[nb][i], 0.f);
      }
      v += __shfl_xor(v, 16, 64);
      v += __shfl_xor(v, 32, 64);
      if (lane < 16) wsum[w][nb * 16 + lane] = v;
    }
    __syncthreads();
    if (tid < kConvCout) {
      const float t = ((wsum[0][tid] + wsum[1][tid]) + wsum[2][tid]) + wsum[3][tid];
      a.sp.partial[((int64_t)r * ntiles + tile) * kConvCout + tid] = t;
    }
    __syncthreads();
  }
  if (!grid_barrier(ctl, xnwg(a), a.spin_ticks, false, xwg(a))) return false;
  const float inv = 1.f / (float)npix;
  for (int i = xwg(a) * kThreads + tid; i < rows * kConvCout; i += xnwg(a) * kThreads) {
    const int r = i / kConvCout, c = i - r * kConvCout;
    const float* pp = a.sp.partial + (int64_t)r * ntiles * kConvCout + c;
    float t = 0.f;
    for (int q = 0; q < ntiles; ++q) t += pp[(int64_t)q * kConvCout];
    out_f32(&((float*)out)[(int64_t)r * kConvCout + c], t * inv);
  }
  return true;
}

// ------------------------------------------------------------------ gather + score
// One wave per row: the row's query vectors are staged in LDS. When the table width
// is a multiple of 8 (its rows are then 16-byte aligned), each quarter wave takes one
// id: its 16 lanes read the table row in contiguous 16-byte pieces once and score it
// against every head. Other widths: each lane computes whole dot products (in order
// over d) for the (head, id) outputs lane, lane + 64, ...
constexpr int kScoreMaxQ = 1024;

__device__ void exec_gather_score(const WorkerArgs& a, WorkerCtl* ctl, const BatchRows& br, int rows, uint8_t* out) {
  __shared__ __attribute__((aligned(16))) float q_s[kWaves][kScoreMaxQ];   // read as float4
  const int qdim = a.sp.dims[0], dim = a.sp.dims[1], n_ids = a.sp.dims[2];
  const int heads = qdim / dim;
  const int64_t trows = a.sp.k;
  const __half* T = (const __half*)a.sp.w[0];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float* Y = (float*)out;
  for (int r = xwg(a) * kWaves + w; r < rows; r += xnwg(a) * kWaves) {
    const float* q = (const float*)br.row(r);
    const int32_t* ids = (const int32_t*)br.bd->rowside[r];
    for (int i = lane; i < qdim; i += 64) q_s[w][i] = q[i];
    wave_lds_sync();
    const int g = lane >> 4, sl = lane & 15;
    if (dim % 8 == 0 && dim <= 128) {
      // rows of at most 128 values: a quarter wave per id, lane s holding piece s (8
      // values) of the row; the rows of 8 ids per quarter wave (32 per wave) are loaded
      // before any is scored. Per head, the lane adds its 8 products in order and the 16
      // lanes' sums are added by a fixed butterfly: one summation order per score, the
      // same as the wider rows' path below
      for (int j0 = 0; j0 < n_ids; j0 += 32) {
        int idv[8];
#pragma unroll
        for (int b = 0; b < 8; ++b) {
          const int j = j0 + 4 * b + g;
          idv[b] = j < n_ids ? ids[j] : -1;
        }
        uint4 tv[8];
#pragma unroll
        for (int b = 0; b < 8; ++b)
          tv[b] = (idv[b] >= 0 && idv[b] < trows && sl * 8 < dim) ? gld16(T + (int64_t)idv[b] * dim + sl * 8)
                                                               : make_uint4(0u, 0u, 0u, 0u);
        for (int h = 0; h < heads; ++h) {
          float qv[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
          if (sl * 8 < dim) {
            const float4 qa = *(const float4*)(q_s[w] + h * dim + sl * 8), qb = *(const float4*)(q_s[w] + h * dim + sl * 8 + 4);
            qv[0] = qa.x; qv[1] = qa.y; qv[2] = qa.z; qv[3] = qa.w; qv[4] = qb.x; qv[5] = qb.y; qv[6] = qb.z; qv[7] = qb.w;
          }
#pragma unroll
          for (int b = 0; b < 8; ++b) {
            const uint32_t u[4] = {tv[b].x, tv[b].y, tv[b].z, tv[b].w};
            float acc = 0.f;
            if (sl * 8 < dim) {
#pragma unroll
              for (int e = 0; e < 8; ++e)
                acc = fmaf(qv[e], __half2float(__ushort_as_half((unsigned short)(u[e >> 1] >> (16 * (e & 1))))), acc);
            }
#pragma unroll
            for (int m = 8; m > 0; m >>= 1) acc += __shfl_xor(acc, m, 64);
            const int j = j0 + 4 * b + g;
            if (sl == 0 && j < n_ids)
              out_f32(&Y[((int64_t)r * heads + h) * n_ids + j], (idv[b] >= 0 && idv[b] < trows) ? acc : 0.f);
          }
        }
      }
    } else if (dim % 8 == 0) {
      // wider rows: lane s holds pieces s, s + 16, ... of one id's row for all heads,
      // adds them in order, then the same butterfly
      for (int j0 = 0; j0 < n_ids; j0 += 4) {
        const int j = j0 + g;
        const int id = j < n_ids ? ids[j] : -1;
        const bool in = id >= 0 && id < trows;
        uint4 tv[kScoreMaxQ / 128];
#pragma unroll
        for (int p = 0; p < kScoreMaxQ / 128; ++p) {
          const int d0 = p * 128 + sl * 8;
          tv[p] = (in && d0 < dim) ? gld16(T + (int64_t)id * dim + d0) : make_uint4(0u, 0u, 0u, 0u);
        }
        for (int h = 0; h < heads; ++h) {
          const float* qh = q_s[w] + h * dim;
          float acc = 0.f;
#pragma unroll
          for (int p = 0; p < kScoreMaxQ / 128; ++p) {
            const int d0 = p * 128 + sl * 8;
            if (d0 < dim) {
              const float4 qa = *(const float4*)(qh + d0), qb = *(const float4*)(qh + d0 + 4);
              const uint32_t u[4] = {tv[p].x, tv[p].y, tv[p].z, tv[p].w};
              const float qv[8] = {qa.x, qa.y, qa.z, qa.w, qb.x, qb.y, qb.z, qb.w};
#pragma unroll
              for (int e = 0; e < 8; ++e)
                acc = fmaf(qv[e], __half2float(__ushort_as_half((unsigned short)(u[e >> 1] >> (16 * (e & 1))))), acc);
            }
          }
#pragma unroll
          for (int m = 8; m > 0; m >>= 1) acc += __shfl_xor(acc, m, 64);
          if (sl == 0 && j < n_ids) out_f32(&Y[((int64_t)r * heads + h) * n_ids + j], in ? acc : 0.f);
        }
      }
    } else {
      // other widths: one (head, id) per lane, the row walked in order
      for (int o = lane; o < heads * n_ids; o += 64) {
        const int h = o / n_ids, j = o - h * n_ids;
        const int id = ids[j];
        float acc = 0.f;
        if (id >= 0 && id < trows) {
          const __half* tr = T + (int64_t)id * dim;
          const float* qh = q_s[w] + h * dim;
          for (int d = 0; d < dim; ++d) acc = fmaf(qh[d], __half2float(tr[d]), acc);
        }
        out_f32(&Y[(int64_t)r * heads * n_ids + o], acc);
      }
    }
    wave_lds_sync();
  }
}

// ------------------------------------------------------------------ artifact stages
// The synthetic microservices of the paper's artifact suite (Section III-B, Section
// VIII-E): a PCIe-intensive, a compute-intensive and a memory-intensive stage, each
// with a tunable intensity. Rows are D = dims[0] 32-bit words (a multiple of 1024).
//
// PCIe / memory: the row's block (dims[1] words, a multiple of D, block number
// in[0] mod (k / dims[1])) of a k-word table - pinned host memory read over the
// host link (ARTIFACT_P) or device memory (ARTIFACT_M) - folded into D words by XOR
// (word j of the fold = XOR of block words j, j + D, ...), XORed into the row.
// ARTIFACT_P keeps the words; ARTIFACT_M turns each into a float in [0, 1), its
// top 24 bits times 2^-24. One workgroup per row: its 256 threads read 16 bytes each,
// 4 KiB contiguous per step, 8 steps in flight; XOR needs no fixed order.
//
// Compute: each word w becomes x = 1 + (w >> 9) 2^-23 (a float in [1, 2)), then
// dims[1] times x = x (1 - 2^-11) + 2^-10, a multiply and an add each rounded to
// FP32 (no fused multiply-add), and the row is the floats' bits. One workgroup per
// row, 4 independent chains per thread.
constexpr int kArtWordsPerStep = kThreads * 4;       // 1024 words: one D slice per step

template <bool FLOAT_OUT>
__device__ void exec_artifact_fold(const WorkerArgs& a, const BatchRows& br, int rows, uint8_t* out) {
  const int D = a.sp.dims[0];
  const int64_t bw = a.sp.dims[1], nblocks = (int64_t)a.sp.k / bw;
  const uint32_t* T = (const uint32_t*)a.sp.w[0];
  const int tid = threadIdx.x;
  for (int r = xwg(a); r < rows; r += xnwg(a)) {
    const uint32_t* in = (const uint32_t*)br.row(r);
    const uint32_t* blk = T + (int64_t)(in[0] % (uint64_t)nblocks) * bw;
    for (int j0 = 0; j0 < D; j0 += kArtWordsPerStep) {
      u32x4_t acc = {0u, 0u, 0u, 0u};
      const int64_t steps = bw / D;
      int64_t t = 0;
      for (; t + 8 <= steps; t += 8) {
        u32x4_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = *(const u32x4_t*)(blk + (t + u) * D + j0 + 4 * tid);
#pragma unroll
        for (int u = 0; u < 8; ++u) acc ^= v[u];
      }
      for (; t < steps; ++t) acc ^= *(const u32x4_t*)(blk + t * D + j0 + 4 * tid);
      const u32x4_t x = *(const u32x4_t*)(in + j0 + 4 * tid) ^ acc;
      if constexpr (FLOAT_OUT) {
        float4 f;
        f.x = (float)(x.x >> 8) * 0x1p-24f;
        f.y = (float)(x.y >> 8) * 0x1p-24f;
        f.z = (float)(x.z >> 8) * 0x1p-24f;
        f.w = (float)(x.w >> 8) * 0x1p-24f;
        u32x4_t q;
        __builtin_memcpy(&q, &f, 16);
        out_u32x4(out, (uint32_t)(((int64_t)r * D + j0 + 4 * tid) * 4), q);
      } else {
        out_u32x4(out, (uint32_t)(((int64_t)r * D + j0 + 4 * tid) * 4), x);
      }
    }
  }
}

__device__ void exec_artifact_compute(const WorkerArgs& a, const BatchRows& br, int rows, uint8_t* out) {
  // two roundings per iteration, as defined: the product and the sum are not fused
#pragma clang fp contract(off)
  const int D = a.sp.dims[0], n = a.sp.dims[1];
  const float mul = 1.0f - 0x1p-11f, add = 0x1p-10f;
  const int tid = threadIdx.x;
  for (int r = xwg(a); r < rows; r += xnwg(a)) {
    const uint32_t* in = (const uint32_t*)br.row(r);
    for (int j0 = 0; j0 < D; j0 += kArtWordsPerStep) {
      const u32x4_t w = *(const u32x4_t*)(in + j0 + 4 * tid);
      float x0 = __uint_as_float((w.x >> 9) | 0x3F800000u), x1 = __uint_as_float((w.y >> 9) | 0x3F800000u);
      float x2 = __uint_as_float((w.z >> 9) | 0x3F800000u), x3 = __uint_as_float((w.w >> 9) | 0x3F800000u);
      for (int i = 0; i < n; ++i) {
        x0 = x0 * mul + add;
        x1 = x1 * mul + add;
        x2 = x2 * mul + add;
        x3 = x3 * mul + add;
      }
      out_u32x4(out, (uint32_t)(((int64_t)r * D + j0 + 4 * tid) * 4),
                (u32x4_t){__float_as_uint(x0), __float_as_uint(x1), __float_as_uint(x2), __float_as_uint(x3)});
    }
  }
}

// ------------------------------------------------------------------ side bytes
// Copies every row's side bytes from the input to the output slot's side plane.
__device__ __forceinline__ void copy_side(const WorkerArgs& a, const BatchDesc* bd, int rows) {
  if (a.side_bytes <= 0 || a.out_kind != kOutRing) return;
  uint8_t* dst = (uint8_t*)bd->out_hdr + a.out_side_off;
  const int words = a.side_bytes >> 2;
  for (int i = xwg(a) * kThreads + threadIdx.x; i < rows * words; i += xnwg(a) * kThreads) {
    const int r = i / words, wd = i - r * words;
    out_u32(&((uint32_t*)(dst + (int64_t)r * a.side_bytes))[wd], ((const uint32_t*)bd->rowside[r])[wd]);
  }
}

// ------------------------------------------------------------------ stage dispatch
template <int KIND>
__device__ __forceinline__ bool exec_stage(const WorkerArgs& a, WorkerCtl* ctl, const BatchRows& br, int rows,
                                           uint8_t* out) {
  if constexpr (KIND == CAMELOT_STAGE_GEMM_RELU) { exec_gemm_relu(a, ctl, br, rows, out); return true; }
  if constexpr (KIND == CAMELOT_STAGE_GEMM_ARGMAX) { exec_gemm_argmax(a, ctl, br, rows); return true; }
  if constexpr (KIND == CAMELOT_STAGE_LOGMEL) { exec_logmel(a, ctl, br, rows, out); return true; }
  if constexpr (KIND == CAMELOT_STAGE_MLP_BF16) { return exec_mlp(a, ctl, br, rows, out); }
  if constexpr (KIND == CAMELOT_STAGE_TOPK) { exec_topk(a, ctl, br, rows); return true; }
  if constexpr (KIND == CAMELOT_STAGE_GATHER) { exec_gather(a, ctl, br, rows, out); return true; }
  if constexpr (KIND == CAMELOT_STAGE_CONV_POOL) { return exec_conv_pool(a, ctl, br, rows, out); }
  if constexpr (KIND == CAMELOT_STAGE_GATHER_SCORE) { exec_gather_score(a, ctl, br, rows, out); return true; }
  if constexpr (KIND == CAMELOT_STAGE_ARTIFACT_P) { exec_artifact_fold<false>(a, br, rows, out); return true; }
  if constexpr (KIND == CAMELOT_STAGE_ARTIFACT_C) { exec_artifact_compute(a, br, rows, out); return true; }
  if constexpr (KIND == CAMELOT_STAGE_ARTIFACT_M) { exec_artifact_fold<true>(a, br, rows, out); return true; }
  return false;
}

// ------------------------------------------------------------------ control side
// Ring slot states: 0 free (never used), 2*seq+1 full with batch seq,
// 2*seq+2 consumed after batch seq.
// Doorbell polling: relaxed loads (no cache invalidation per poll); the caller
// issues one acquire fence once the awaited value is seen.
__device__ __forceinline__ uint64_t ring_load(const uint64_t* p, bool sys) {
  return sys ? __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)
             : __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void ring_acquire(bool sys) {
  if (sys) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
  else __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}
__device__ __forceinline__ void ring_store(uint64_t* p, uint64_t v, bool sys) {
  if (sys) st_release_sys(p, v); else st_release_agent(p, v);
}

struct Acq {
  int status;      // 0 ok (batch ready), else a WorkerStatus to exit with
  int nreq;
  int rows;
};

// Polling helper: true when the host asked to stop (checked every 16th call).
__device__ __forceinline__ bool host_stop(const WorkerArgs& a, uint32_t& polls) {
  if ((++polls & 15u) != 0) return false;
  return __hip_atomic_load(&a.hctl->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0;
}

// Status of a one-poll acquisition that found the batch not ready (never published).
constexpr int kAcqNotReady = -1;

// Stage 0: form a batch from the ingest (wave 0 of the control workgroup), starting at
// ingest record c. Requests are taken whole, in order, while the rows fit in
// max_batch; the batch starts when batch_target rows wait, when the next waiting
// request does not fit, or when the oldest waited batch_timeout. Writes the chosen
// requests into LDS arrays. try_only: one pass, kAcqNotReady if no batch starts.
__device__ __forceinline__ Acq acquire_ingest(const WorkerArgs& a, uint64_t c, uint64_t t0, bool try_only, uint64_t* s_id,
                              uint64_t* s_tarr, uint32_t* s_rows, const uint8_t** s_ptr) {
  const int lane = threadIdx.x & 63;
  // replay arrival times are relative to the epoch t0; host ones are absolute
  const uint64_t base = a.in_kind == kInHost ? 0 : t0;
  const uint64_t t_wait0 = now_ticks();
  uint32_t polls = 0;
  const bool host = a.in_kind == kInHost;
  for (;;) {
    uint64_t avail;
    if (host) {
      const uint64_t head = ld_acquire_sys(&a.hctl->ingest_head);   // one PCIe read per poll
      avail = head > c ? head - c : 0;
    } else {
      avail = (uint64_t)a.n_ingest > c ? (uint64_t)a.n_ingest - c : 0;
    }
    const uint64_t now = now_ticks();
    int taken = 0, rows = 0, full = 0;
    uint64_t first_tarr = 0;
    // up to two 64-request chunks (a batch holds at most kMaxBatch >= requests)
    for (int chunk = 0; chunk < 2 && !full; ++chunk) {
      const uint64_t i = (uint64_t)(chunk * 64 + lane);
      const bool valid = i < avail && taken == chunk * 64;
      IngestRec rec = {};
      if (valid) {
        const uint64_t r = c + i;
        rec = a.ingest[host ? (r % (uint64_t)a.n_ingest) : r];
        rec.t_arr += base;
      }
      const bool arrived = valid && (host || rec.t_arr <= now);
      // prefix of arrived requests
      const uint64_t nb = __ballot(!arrived);
      const int first_gap = nb ? __builtin_ctzll(nb) : 64;
      int v = (arrived && lane < first_gap) ? (int)rec.rows : 0;
      int cum = v;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const int t = __shfl_up(cum, d, 64);
        if (lane >= d) cum += t;
      }
      const bool fits = arrived && lane < first_gap && rows + cum <= a.max_batch;
      const uint64_t fm = __ballot(fits);
      const int nfit = fm ? 64 - __builtin_clzll(fm) : 0;  // fits is a prefix
      if (fits) {
        const int q = taken + lane;
        s_id[q] = rec.id;
        s_tarr[q] = rec.t_arr;
        s_rows[q] = rec.rows;
        s_ptr[q] = a.ingest_payload + rec.payload_off;
      }
      if (chunk == 0) first_tarr = __shfl(rec.t_arr, 0, 64);
      const int add_rows = __shfl(cum, nfit > 0 ? nfit - 1 : 0, 64);
      if (nfit > 0) rows += add_rows;
      taken += nfit;
      // a waiting request that does not fit makes the batch full
      if (nfit < first_gap) full = 1;
      if (first_gap < 64) break;
    }
    if (taken > 0) {
      const bool timeout = (int64_t)(now - first_tarr) >= a.batch_timeout_ticks;
      if (full || rows >= a.batch_target || rows >= a.max_batch || timeout) {
        return Acq{0, taken, rows};
      }
    }
    if (try_only) return Acq{kAcqNotReady, 0, 0};
    if (host_stop(a, polls)) return Acq{kStatusStopped, 0, 0};
    if ((int64_t)(now - t_wait0) > a.idle_ticks) return Acq{kStatusIdleExit, 0, 0};
    __builtin_amdgcn_s_sleep(2);
  }
}

// Stages > 0: wait until input slot seq is full and, for a ring output, output slot
// seq is free: both doorbells in each poll, one acquire once both are seen
// (try_only: one poll). Returns 0 or the status to exit with.
__device__ __forceinline__ int acquire_ring_slots(const WorkerArgs& a, uint64_t seq, bool try_only) {
  const bool in_sys = a.in_state_sys != 0, out_sys = a.out_state_sys != 0;
  const bool ring_out = a.out_kind == kOutRing;
  const uint64_t* in_p = &a.in_state[seq % (uint64_t)a.in_depth];
  const uint64_t want_in = 2 * seq + 1;
  const uint64_t* out_p = ring_out ? &a.out_state[seq % (uint64_t)a.out_depth] : nullptr;
  const uint64_t want_out = !ring_out || seq < (uint64_t)a.out_depth ? 0 : 2 * (seq - a.out_depth) + 2;
  const uint64_t t_wait0 = now_ticks();
  uint32_t polls = 0;
  for (;;) {
    const uint64_t vi = ring_load(in_p, in_sys);
    const uint64_t vo = ring_out ? ring_load(out_p, out_sys) : 0;
    if (vi == want_in && vo == want_out) {
      ring_acquire(in_sys || (ring_out && out_sys));
      return 0;
    }
    if (try_only) return kAcqNotReady;
    if (host_stop(a, polls)) return kStatusStopped;
    if ((int64_t)(now_ticks() - t_wait0) > a.idle_ticks) return kStatusIdleExit;
    __builtin_amdgcn_s_sleep(1);
  }
}

// Wait until the output can take batch seq of `rows` rows (try_only: one poll).
// Egress space is counted from egress_head, the rows of every batch formed so far
// (formation reserves them); tail_seen is the host's tail as last read.
__device__ __forceinline__ int acquire_output(const WorkerArgs& a, uint64_t egress_head, uint64_t& tail_seen,
                                              uint64_t seq, int rows, bool try_only) {
  const uint64_t t_wait0 = now_ticks();
  uint32_t polls = 0;
  for (;;) {
    bool ok;
    if (a.out_kind == kOutRing) {
      const uint64_t slot = seq % (uint64_t)a.out_depth;
      const uint64_t want = seq < (uint64_t)a.out_depth ? 0 : 2 * (seq - a.out_depth) + 2;
      ok = ring_load(&a.out_state[slot], a.out_state_sys != 0) == want;
    } else {
      // the tail last read is a lower bound of the host's (it only grows): a PCIe read
      // only when that bound leaves too little room; space already seen was acquired
      // when it was read
      if (egress_head + (uint64_t)rows - tail_seen <= (uint64_t)a.egress_cap) return 0;
      const uint64_t tail = __hip_atomic_load(&a.hctl->egress_tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      tail_seen = tail;
      ok = egress_head + (uint64_t)rows - tail <= (uint64_t)a.egress_cap;
    }
    if (ok) {
      ring_acquire(a.out_kind != kOutRing || a.out_state_sys != 0);
      return 0;
    }
    if (try_only) return kAcqNotReady;
    if (host_stop(a, polls)) return kStatusStopped;
    if ((int64_t)(now_ticks() - t_wait0) > a.idle_ticks) return kStatusIdleExit;
    __builtin_amdgcn_s_sleep(1);
  }
}

// ------------------------------------------------------------------ one-shot / profiling kernel
// Runs the stage's compute `reps` times back to back on a fixed input with the
// same grid and the same code as the persistent worker (used for parity checks
// and for the solo profiling table).
template <int KIND>
__global__ __launch_bounds__(kThreads, kMinWgPerCuResident) void stage_bench(WorkerArgs a) {
  WorkerCtl* ctl = a.ctl;
  const int tid = threadIdx.x;
  if (blockIdx.x == 0)
    for (int i = tid; i < a.bench_rows; i += kThreads) {
      ctl->dd[0].rowptr[i] = a.bench_in + (int64_t)i * a.in_row_stride;
      ctl->dd[0].rowside[i] = ctl->dd[0].rowptr[i] + a.sp.in_row_bytes;
    }
  if (!grid_barrier(ctl, gridDim.x, a.spin_ticks)) return;
  const uint64_t t0 = now_ticks();
  int rep = 0;
  while (rep < a.bench_reps) {
    if (!exec_stage<KIND>(a, ctl, batch_rows(a, &ctl->dd[0], 0), a.bench_rows, a.bench_out)) return;
    ++rep;
    // duration mode: workgroup 0 decides for the whole grid, published by the barrier;
    // two slots by parity so a fast workgroup 0 never overwrites a decision that a
    // slow workgroup has not read yet
    if (blockIdx.x == 0 && tid == 0)
      ctl->bench_stop[rep & 1] = (a.bench_ticks > 0 && (int64_t)(now_ticks() - t0) >= a.bench_ticks) ? 1u : 0u;
    if (!grid_barrier(ctl, gridDim.x, a.spin_ticks)) return;
    if (ctl->bench_stop[rep & 1]) break;
  }
  if (blockIdx.x == 0 && tid == 0) {
    ctl->ticks_bench = now_ticks() - t0;
    ctl->reps_bench = (uint64_t)rep;
  }
}

// ------------------------------------------------------------------ worker kernel
// Compute workgroups wait here for the control workgroup's broadcast of batch `want`
// (bounded; an abort raised anywhere ends the wait).
__device__ __forceinline__ bool wait_go(WorkerCtl* ctl, uint32_t want, int64_t spin_ticks) {
  __shared__ int s_go;
  if (threadIdx.x == 0) {
    int ok = 1;
    const uint64_t t0 = now_ticks();
    uint32_t polls = 0;
    const uint32_t* gp = &ctl->go[blockIdx.x & 7u][0];
    while (__hip_atomic_load(const_cast<uint32_t*>(gp), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != want) {
      ++polls;
      if ((polls & 15u) == 0 && __hip_atomic_load(&ctl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        ok = 0;
        break;
      }
      if ((int64_t)(now_ticks() - t0) > spin_ticks) {
        __hip_atomic_store(&ctl->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      poll_backoff(polls);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    s_go = ok;
  }
  __syncthreads();
  // every wave acquires too: the descriptor slot is small and re-read every second
  // batch, so stale copies of it can survive in a reader's caches
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return s_go != 0;
}

// What the control workgroup stages in LDS for one batch while forming it.
struct BatchLds {
  uint64_t id[kMaxBatch];               // request ids
  uint64_t tarr[kMaxBatch];             // request arrival ticks
  uint32_t rows[kMaxBatch];             // rows per request
  const uint8_t* ptr[kMaxBatch];        // stage 0: first payload row of each request
  uint32_t rbase[kMaxBatch + 1];        // first row of each request in the batch
  uint64_t t_stage[2 * kMaxStages];     // stage timestamps carried by the input slot
  uint64_t red[2][kWaves];              // per-wave id checksums (sum, xor)
  uint64_t cursor;                      // stage 0: next ingest record not in a batch
  uint64_t egress_base;                 // terminal stage: first egress row of the batch
  uint64_t egress_head;                 // terminal stage: egress rows of the batches formed
  uint64_t egress_tail_seen;            // terminal stage: the host's egress tail as last read
  int acq[3];                           // status, requests, rows
};

// Formation of batch seq by all threads of the control workgroup: acquire its input (ingest
// requests, or the full ring slot seq) and its output space, then stage the
// requests, their row offsets, the input's stage timestamps and the id checksums
// in LDS. Stage 0 takes the requests (advances the ingest cursor) and a terminal
// stage reserves the egress rows only when the batch is formed. try_only: one poll,
// kAcqNotReady when the batch is not ready, and then nothing is taken.
// Returns 0 when the batch is staged, else the status.
__device__ __forceinline__ int form_batch(const WorkerArgs& a, WorkerCtl* ctl, uint64_t seq, uint64_t t0, bool try_only,
                          BatchLds& s) {
  const int tid = threadIdx.x;
  const bool first = a.in_kind != kInRing;     // takes requests from the ingest
  int nreq;
  if (first) {
    if (tid < 64) {
      Acq q = acquire_ingest(a, s.cursor, t0, try_only, s.id, s.tarr, s.rows, s.ptr);
      if (q.status == 0 && tid == 0)
        q.status = acquire_output(a, s.egress_head, s.egress_tail_seen, seq, q.rows, try_only);
      if (tid == 0) { s.acq[0] = q.status; s.acq[1] = q.nreq; s.acq[2] = q.rows; }
    }
    if (tid < 2 * kMaxStages) s.t_stage[tid] = 0;
    __syncthreads();
    if (s.acq[0] != 0) return s.acq[0];
    nreq = s.acq[1];
  } else {
    if (tid == 0) s.acq[0] = acquire_ring_slots(a, seq, try_only);
    __syncthreads();
    if (s.acq[0] != 0) return s.acq[0];
    // every wave reads the slot header: every wave acquires
    if (a.in_state_sys || (a.out_kind == kOutRing && a.out_state_sys)) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
    else __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");

    // the whole header in one round of loads: the counts, the stage times and every
    // request entry (those past n_req are not used)
    const SlotHeader* ih = (const SlotHeader*)(a.in_ring + (seq % (uint64_t)a.in_depth) * (uint64_t)a.in_stride);
    const int hreq = (int)ih->n_req, hrows = (int)ih->n_rows;
    for (int q = tid; q < kMaxBatch; q += kThreads) {
      s.id[q] = ih->req_id[q];
      s.tarr[q] = ih->req_tarr[q];
      s.rows[q] = ih->req_rows[q];
    }
    if (tid < 2 * kMaxStages) s.t_stage[tid] = ih->t_stage[tid];
    __syncthreads();       // every thread has read s.acq[0]
    if (tid == 0) {
      // a terminal stage's egress space needs the row count (usually no round trip)
      s.acq[0] = a.out_kind == kOutEgress
                     ? acquire_output(a, s.egress_head, s.egress_tail_seen, seq, hrows, try_only) : 0;
      s.acq[1] = hreq;
      s.acq[2] = hrows;
    }
    __syncthreads();
    if (s.acq[0] != 0) return s.acq[0];
    nreq = hreq;
  }
  if (tid < 64) {
    // first row of each request: exclusive prefix sum of the row counts, 64 at a time
    uint32_t carry = 0;
    for (int b = 0; b < nreq; b += 64) {
      const int q = b + tid;
      const uint32_t v = q < nreq ? s.rows[q] : 0u;
      uint32_t inc = v;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const uint32_t t = __shfl_up(inc, d, 64);
        if (tid >= d) inc += t;
      }
      if (q < nreq) s.rbase[q] = carry + inc - v;
      carry += __shfl(inc, 63, 64);
    }
    if (tid == 0) {
      s.rbase[nreq] = carry;
      if (first) s.cursor += (uint64_t)nreq;
      if (a.out_kind == kOutEgress) {
        s.egress_base = s.egress_head;
        s.egress_head += (uint64_t)s.acq[2];
      }
    }
  }
  // id checksums of the requests of this batch
  uint64_t hs = 0, hx = 0;
  for (int q = tid; q < nreq; q += kThreads) {
    const uint64_t h = id_hash(s.id[q]);
    hs += h;
    hx ^= h;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    hs += __shfl_xor(hs, off, 64);
    hx ^= __shfl_xor(hx, off, 64);
  }
  if ((tid & 63) == 0) { s.red[0][tid >> 6] = hs; s.red[1][tid >> 6] = hx; }
  __syncthreads();
  return 0;
}

// A formation try while a batch runs only this long before its expected end (ticks).
constexpr int64_t kTryMarginTicks = 500;

// What the publication of a batch needs (control workgroup).
struct BatchPub {
  uint64_t seq, hs, hx, t_start, t_top, t_end, ingest_end, egress_end;
  int rows;
};

// Persistent worker, control side (the last workgroup). Per batch: form it (or take the
// one formed early), write its descriptor and broadcast it; then, while the compute
// workgroups run the batch, try to form the next one (seq + n_inst) and wait until
// every compute workgroup has counted the batch done. The batch is published
// (output doorbell, input slot release or ingest tail, egress head, counters) right
// after the next batch's broadcast, or before waiting for input when the next batch
// is not ready. Acquisition, staging and publication thus run beside the stage's
// compute; between two batches remain the descriptor and the broadcast.
// side_ptrs: the stage reads each row's side bytes.
__device__ __forceinline__ void worker_control(const WorkerArgs& a, bool side_ptrs) {
  WorkerCtl* ctl = a.ctl;
  const int tid = threadIdx.x;
  // the stage's place in the timestamps (after the stages of upstream processes);
  // the first stage of this pipeline takes requests from the ingest, the others a ring
  const int si = a.stage_index;
  const bool first = a.in_kind != kInRing;
  const int nx = (int)gridDim.x - 1;              // compute workgroups
  const int ng = nx < 8 ? nx : 8;                 // their groups (index mod 8)

  __shared__ BatchLds s;
  __shared__ uint64_t s_t0;
  // running counters (thread 0). A terminal stage publishes them with each batch,
  // before its results; the others every 16th batch (their stores to host memory
  // would hold up the next loads of the thread that issued them), before waiting for
  // input, and at exit (acc_dirty: not published yet)
  __shared__ uint64_t acc_sum, acc_xor, acc_batches, acc_rows, acc_busy, acc_wait;
  __shared__ int acc_dirty;
  __shared__ uint32_t done_base[8];               // the done counters at start
  __shared__ int s_flag;
  __shared__ int64_t s_dur;                       // how long the last batch ran (ticks)
  __shared__ BatchPub pb;                         // the batch awaiting publication
  auto publish_counters = [&]() {
    st_relaxed_sys(&a.pub->id_sum[a.worker_index], acc_sum);
    st_relaxed_sys(&a.pub->id_xor[a.worker_index], acc_xor);
    st_relaxed_sys(&a.pub->rows[a.worker_index], acc_rows);
    st_relaxed_sys(&a.pub->busy_ticks[a.worker_index], acc_busy);
    st_relaxed_sys(&a.pub->wait_ticks[a.worker_index], acc_wait);
    st_relaxed_sys(&a.pub->batches[a.worker_index], acc_batches);
    acc_dirty = 0;
  };
  // publication of batch pb (thread 0): one release fence for the output doorbell
  // and the input slot release
  auto publish_batch = [&]() {
    const uint64_t q = pb.seq;
    const bool sys = a.out_kind == kOutEgress || a.out_state_sys != 0 || a.in_state_sys != 0;
    if (a.out_kind == kOutRing) {
      SlotHeader* oh = (SlotHeader*)(a.out_ring + (q % (uint64_t)a.out_depth) * (uint64_t)a.out_stride);
      oh->t_stage[2 * si + 1] = pb.t_end;
      // host-staged boundary: the relay reads the row count next to the state word
      if (a.out_state_sys) st_relaxed_sys(&a.out_state[a.out_depth + q % (uint64_t)a.out_depth], (uint64_t)pb.rows);
    }
    acc_sum += pb.hs;
    acc_xor ^= pb.hx;
    acc_batches += 1;
    acc_rows += (uint64_t)pb.rows;
    acc_busy += pb.t_end - pb.t_start;
    acc_wait += pb.t_start - pb.t_top;
    acc_dirty = 1;
    if (a.out_kind == kOutEgress) publish_counters();     // ordered before the results by the fence
    if (sys) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
    else __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (a.out_kind == kOutRing) {
      uint64_t* p = &a.out_state[q % (uint64_t)a.out_depth];
      if (a.out_state_sys) st_relaxed_sys(p, 2 * q + 1);
      else __hip_atomic_store(p, 2 * q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      st_relaxed_sys(&a.pub->egress_head, pb.egress_end);
    }
    if (first) {
      st_relaxed_sys(&a.pub->ingest_tail, pb.ingest_end);
    } else {
      uint64_t* p = &a.in_state[q % (uint64_t)a.in_depth];
      if (a.in_state_sys) st_relaxed_sys(p, 2 * q + 2);
      else __hip_atomic_store(p, 2 * q + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  };

  if (tid == 0) {
    s_t0 = now_ticks();
    s.cursor = ctl->ingest_cursor;
    s.egress_head = ctl->egress_head;
    s.egress_tail_seen = ctl->egress_tail_seen;
    acc_sum = ctl->sum_acc;
    acc_xor = ctl->xor_acc;
    acc_batches = ctl->batches_acc;
    acc_rows = ctl->rows_acc;
    acc_busy = ctl->busy_acc;
    acc_wait = ctl->wait_acc;
    acc_dirty = 0;
    s_dur = 0;
    // the compute workgroups count a batch only after its broadcast
    for (int g = 0; g < 8; ++g) done_base[g] = __hip_atomic_load(&ctl->done[g][0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (first) st_relaxed_sys(&a.pub->t0, s_t0);
    st_relaxed_sys(&a.pub->started[a.worker_index], 1);
  }
  __syncthreads();
  uint64_t seq = ctl->next_seq;
  uint32_t issued = 0;            // batches broadcast by this launch
  int exit_status = kStatusOk;
  bool pending = false;           // batch seq is already formed and staged
  bool unpublished = false;       // pb holds a finished batch not yet published
  bool desc_ready = false;        // batch seq's descriptor is already written
  // The descriptor of batch q (staged in s) into slot `slot` (the batch's number in
  // the launch mod 2), and its output slot's header; st != 0: only the stop.
  auto write_desc = [&](uint32_t slot, uint64_t q, int st) {
    BatchDesc& d = ctl->dd[slot];
    if (st == 0) {
      const int nreq = s.acq[1], rows = s.acq[2];
      // per-row descriptors: input row pointers (ingest), side bytes, and the
      // request of each row (egress records)
      const uint8_t* in_payload = !first ? a.in_ring + (q % (uint64_t)a.in_depth) * (uint64_t)a.in_stride +
                                               kSlotHeaderBytes
                                         : nullptr;
      const uint8_t* in_hdr = !first ? in_payload - kSlotHeaderBytes : nullptr;
      for (int r = tid; r < nreq; r += kThreads) {
        for (uint32_t j = 0; j < s.rows[r]; ++j) {
          const uint32_t row = s.rbase[r] + j;
          const uint8_t* rp = !first ? in_payload + (int64_t)row * a.sp.in_row_bytes
                                     : s.ptr[r] + (int64_t)j * a.in_row_stride;
          if (first) d.rowptr[row] = rp;
          if (side_ptrs)
            d.rowside[row] = !first ? in_hdr + a.in_side_off + (int64_t)row * a.side_bytes
                                    : rp + a.sp.in_row_bytes;
          if (a.out_kind == kOutEgress) {
            d.row_id[row] = s.id[r];
            d.row_idx[row] = j;
            d.row_tarr[row] = s.tarr[r];
          }
        }
      }
      // this stage's start time is filled in at the broadcast
      if (tid < 2 * kMaxStages && tid != 2 * si) d.t_stage[tid] = s.t_stage[tid];
      if (a.out_kind == kOutRing) {
        SlotHeader* oh = (SlotHeader*)(a.out_ring + (q % (uint64_t)a.out_depth) * (uint64_t)a.out_stride);
        for (int r = tid; r < nreq; r += kThreads) {
          oh->req_id[r] = s.id[r];
          oh->req_tarr[r] = s.tarr[r];
          oh->req_rows[r] = s.rows[r];
        }
        if (tid < 2 * kMaxStages && tid != 2 * si) oh->t_stage[tid] = s.t_stage[tid];
        if (tid == 0) {
          oh->seq = q;
          oh->n_req = (uint32_t)nreq;
          oh->n_rows = (uint32_t)rows;
          d.out = (uint8_t*)oh + kSlotHeaderBytes;
          d.out_hdr = oh;
        }
      } else if (tid == 0) {
        d.egress_base = s.egress_base;
        d.out = nullptr;
      }
      if (tid == 0) d.rows = (uint32_t)rows;
    }
    if (tid == 0) d.stop = (uint32_t)st;
  };
  for (;;) {
    const uint64_t t_top = now_ticks();
    int st = pending ? 0 : kAcqNotReady;
    for (int attempt = 0; st == kAcqNotReady; ++attempt) {
      if (attempt == 1) {
        // about to wait for input: what is finished reaches the consumers and the host
        if (tid == 0) {
          if (unpublished) publish_batch();
          if (acc_dirty) publish_counters();
        }
        unpublished = false;
      }
      st = form_batch(a, ctl, seq, s_t0, attempt == 0, s);
    }
    uint64_t t_start = 0;
    const uint32_t slot = issued & 1u;
    if (!desc_ready) write_desc(slot, seq, st);
    pending = false;
    desc_ready = false;
    if (st == 0) {
      // the batch's start time, into its descriptor and its output slot's header
      t_start = now_ticks();
      if (tid == 0) {
        ctl->dd[slot].t_stage[2 * si] = t_start;
        if (a.out_kind == kOutRing)
          ((SlotHeader*)(a.out_ring + (seq % (uint64_t)a.out_depth) * (uint64_t)a.out_stride))->t_stage[2 * si] =
              t_start;
      }
    }
    // broadcast: the batch descriptor (or the stop) is in place
    wg_barrier_stores_done();
    if (tid == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      for (int g = 0; g < 8; ++g)
        __hip_atomic_store(&ctl->go[g][0], (uint32_t)(seq + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      // the previous batch, and now and then the counters, after the broadcast
      if (unpublished) publish_batch();
      if (acc_dirty && (acc_batches & 15) == 0) publish_counters();
    }
    unpublished = false;
    if (st != 0) { exit_status = st; break; }
    ++issued;
    // what the publication of this batch will need (staged data of the next batch
    // may overwrite s from here on)
    if (tid == 0) {
      uint64_t hs = 0, hx = 0;
      for (int w = 0; w < kWaves; ++w) { hs += s.red[0][w]; hx ^= s.red[1][w]; }
      pb.seq = seq;
      pb.hs = hs;
      pb.hx = hx;
      pb.rows = s.acq[2];
      pb.t_start = t_start;
      pb.t_top = t_top;
      pb.ingest_end = s.cursor;
      pb.egress_end = s.egress_base + (uint64_t)s.acq[2];
    }
    __syncthreads();
    // while the batch runs: wait until every compute workgroup has counted it done
    // (bounded; an abort ends it), and form the next batch once it is ready, with
    // tries only while the batch is expected to run for a while longer (a try must
    // not hold up noticing the end)
    const uint64_t t_w0 = now_ticks();
    uint32_t polls = 0;
    int f = 0;
    for (;;) {
      if (tid == 0) {
        bool all = true;
        for (int g = 0; g < ng; ++g) {
          const uint32_t members = (uint32_t)(nx - g + 7) >> 3;
          const uint32_t v = __hip_atomic_load(&ctl->done[g][0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (v - done_base[g] != issued * members) all = false;
        }
        int r = all ? 1 : 0;
        if (!all) {
          const int64_t el = (int64_t)(now_ticks() - t_w0);
          if (__hip_atomic_load(&ctl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            r = -1;
          } else if (el > a.spin_ticks) {
            __hip_atomic_store(&ctl->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            r = -1;
          } else if (!pending && el + kTryMarginTicks < s_dur) {
            r = 2;
          } else {
            poll_backoff(++polls);
          }
        }
        s_flag = r;
      }
      __syncthreads();
      f = s_flag;
      __syncthreads();
      if (f != 2 && f != 0) break;
      if (f == 2) {
        pending = form_batch(a, ctl, seq + (uint64_t)a.n_inst, s_t0, true, s) == 0;
        // the next batch's descriptor now, into the other slot (the batch two back,
        // which used it, has finished)
        if (pending) {
          write_desc(issued & 1u, seq + (uint64_t)a.n_inst, 0);
          desc_ready = true;
        }
      }
    }
    if (f < 0) { exit_status = kStatusTimeout; break; }
    if (tid == 0) {
      // the compute workgroups' results (released before they counted) are visible
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      pb.t_end = now_ticks();
      s_dur = (int64_t)(pb.t_end - t_w0);
    }
    unpublished = true;
    seq += (uint64_t)a.n_inst;          // instance j of n takes batches j, j + n, ...
  }
  if (tid == 0) {
    ctl->next_seq = seq;
    ctl->ingest_cursor = s.cursor;
    ctl->egress_head = s.egress_head;
    ctl->egress_tail_seen = s.egress_tail_seen;
    ctl->sum_acc = acc_sum;
    ctl->xor_acc = acc_xor;
    ctl->batches_acc = acc_batches;
    ctl->rows_acc = acc_rows;
    ctl->busy_acc = acc_busy;
    ctl->wait_acc = acc_wait;
    publish_counters();
    st_release_sys(&a.pub->status[a.worker_index], (int32_t)exit_status);
  }
}

// Persistent worker, compute side (the other workgroups, one per CU of the share): wait for the broadcast of each
// batch this instance takes, run the stage on it, make the results visible (system
// scope for results in host memory or slots a DMA copy reads) and count the batch
// done in the group's counter. A stop in the descriptor, an expired wait or a failed
// stage ends the loop (the control workgroup then times out on the counters, or
// sees the abort).
template <int KIND>
__device__ __forceinline__ void worker_compute(const WorkerArgs& a) {
  WorkerCtl* ctl = a.ctl;
  const int tid = threadIdx.x;
  const uint32_t g = (uint32_t)xwg(a) & 7u;
  const bool sys = a.out_kind == kOutEgress || a.out_state_sys != 0;
  uint64_t seq = ctl->next_seq;
  uint32_t c = 0;                 // batches started in this launch: descriptor slot c mod 2
  for (;;) {
    // the control workgroup may wait for input (up to the idle limit) and then for
    // output space
    if (!wait_go(ctl, (uint32_t)(seq + 1), 2 * a.idle_ticks + a.spin_ticks)) break;
    // a host-staged input slot was written by a DMA copy: acquire at system scope
    if (a.in_state_sys) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
    const BatchDesc* bd = &ctl->dd[c & 1u];
    // the descriptor is the same for every lane: kept in scalar registers
    const uint32_t stop = __builtin_amdgcn_readfirstlane(bd->stop);
    if (stop) break;
    const int rows = __builtin_amdgcn_readfirstlane((int)bd->rows);
    const uint64_t outp = (uint64_t)bd->out;
    uint8_t* const out = (uint8_t*)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(outp >> 32)) << 32) |
                                    (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)outp));
    if (!exec_stage<KIND>(a, ctl, batch_rows(a, bd, seq), rows, out)) break;
    copy_side(a, bd, rows);
    // the rows and side bytes were written through: thread 0's release publishes them
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) {
      if (sys) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
      else __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_fetch_add(&ctl->done[g][0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    seq += (uint64_t)a.n_inst;
    ++c;
  }
}

template <int KIND>
__global__ __launch_bounds__(kThreads, kMinWgPerCuResident) void stage_worker(WorkerArgs a) {
  if ((int)blockIdx.x == xnwg(a)) worker_control(a, a.side_bytes > 0 || KIND == CAMELOT_STAGE_GATHER_SCORE);
  else worker_compute<KIND>(a);
}

template __global__ void stage_worker<CAMELOT_STAGE_GEMM_RELU>(WorkerArgs);
template __global__ void stage_worker<CAMELOT_STAGE_GEMM_ARGMAX>(WorkerArgs);
template __global__ void stage_worker<CAMELOT_STAGE_LOGMEL>(WorkerArgs);
template __global__ void stage_worker<CAMELOT_STAGE_MLP_BF16>(WorkerArgs);
template __global__ void stage_worker<CAMELOT_STAGE_TOPK>(WorkerArgs);
template __global__ void stage_worker<CAMELOT_STAGE_GATHER>(WorkerArgs);
template __global__ void stage_bench<CAMELOT_STAGE_GATHER>(WorkerArgs);
template __global__ void stage_worker<CAMELOT_STAGE_GATHER_SCORE>(WorkerArgs);
template __global__ void stage_bench<CAMELOT_STAGE_GATHER_SCORE>(WorkerArgs);
template __global__ void stage_worker<CAMELOT_STAGE_CONV_POOL>(WorkerArgs);
template __global__ void stage_bench<CAMELOT_STAGE_CONV_POOL>(WorkerArgs);
template __global__ void stage_bench<CAMELOT_STAGE_GEMM_RELU>(WorkerArgs);
template __global__ void stage_bench<CAMELOT_STAGE_GEMM_ARGMAX>(WorkerArgs);
template __global__ void stage_bench<CAMELOT_STAGE_LOGMEL>(WorkerArgs);
template __global__ void stage_bench<CAMELOT_STAGE_MLP_BF16>(WorkerArgs);
template __global__ void stage_bench<CAMELOT_STAGE_TOPK>(WorkerArgs);
template __global__ void stage_worker<CAMELOT_STAGE_ARTIFACT_P>(WorkerArgs);
template __global__ void stage_bench<CAMELOT_STAGE_ARTIFACT_P>(WorkerArgs);
template __global__ void stage_worker<CAMELOT_STAGE_ARTIFACT_C>(WorkerArgs);
template __global__ void stage_bench<CAMELOT_STAGE_ARTIFACT_C>(WorkerArgs);
template __global__ void stage_worker<CAMELOT_STAGE_ARTIFACT_M>(WorkerArgs);
template __global__ void stage_bench<CAMELOT_STAGE_ARTIFACT_M>(WorkerArgs);

// Host-side accessor of the kernel entry for a stage kind (bench: one-shot kernel).
const void* worker_kernel(int kind, bool bench) {
  if (bench) {
    switch (kind) {
      case CAMELOT_STAGE_GEMM_RELU: return (const void*)&stage_bench<CAMELOT_STAGE_GEMM_RELU>;
      case CAMELOT_STAGE_GEMM_ARGMAX: return (const void*)&stage_bench<CAMELOT_STAGE_GEMM_ARGMAX>;
      case CAMELOT_STAGE_LOGMEL: return (const void*)&stage_bench<CAMELOT_STAGE_LOGMEL>;
      case CAMELOT_STAGE_MLP_BF16: return (const void*)&stage_bench<CAMELOT_STAGE_MLP_BF16>;
      case CAMELOT_STAGE_TOPK: return (const void*)&stage_bench<CAMELOT_STAGE_TOPK>;
      case CAMELOT_STAGE_GATHER: return (const void*)&stage_bench<CAMELOT_STAGE_GATHER>;
      case CAMELOT_STAGE_GATHER_SCORE: return (const void*)&stage_bench<CAMELOT_STAGE_GATHER_SCORE>;
      case CAMELOT_STAGE_CONV_POOL: return (const void*)&stage_bench<CAMELOT_STAGE_CONV_POOL>;
      case CAMELOT_STAGE_ARTIFACT_P: return (const void*)&stage_bench<CAMELOT_STAGE_ARTIFACT_P>;
      case CAMELOT_STAGE_ARTIFACT_C: return (const void*)&stage_bench<CAMELOT_STAGE_ARTIFACT_C>;
      case CAMELOT_STAGE_ARTIFACT_M: return (const void*)&stage_bench<CAMELOT_STAGE_ARTIFACT_M>;
      default: return nullptr;
    }
  }
  switch (kind) {
    case CAMELOT_STAGE_GEMM_RELU: return (const void*)&stage_worker<CAMELOT_STAGE_GEMM_RELU>;
    case CAMELOT_STAGE_GEMM_ARGMAX: return (const void*)&stage_worker<CAMELOT_STAGE_GEMM_ARGMAX>;
    case CAMELOT_STAGE_LOGMEL: return (const void*)&stage_worker<CAMELOT_STAGE_LOGMEL>;
    case CAMELOT_STAGE_MLP_BF16: return (const void*)&stage_worker<CAMELOT_STAGE_MLP_BF16>;
    case CAMELOT_STAGE_TOPK: return (const void*)&stage_worker<CAMELOT_STAGE_TOPK>;
    case CAMELOT_STAGE_GATHER: return (const void*)&stage_worker<CAMELOT_STAGE_GATHER>;
    case CAMELOT_STAGE_GATHER_SCORE: return (const void*)&stage_worker<CAMELOT_STAGE_GATHER_SCORE>;
    case CAMELOT_STAGE_CONV_POOL: return (const void*)&stage_worker<CAMELOT_STAGE_CONV_POOL>;
    case CAMELOT_STAGE_ARTIFACT_P: return (const void*)&stage_worker<CAMELOT_STAGE_ARTIFACT_P>;
    case CAMELOT_STAGE_ARTIFACT_C: return (const void*)&stage_worker<CAMELOT_STAGE_ARTIFACT_C>;
    case CAMELOT_STAGE_ARTIFACT_M: return (const void*)&stage_worker<CAMELOT_STAGE_ARTIFACT_M>;
    default: return nullptr;
  }
}
}  // namespace camelot
