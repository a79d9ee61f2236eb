// Shared host/device definitions of the Camelot runtime: ring slot layout, worker
// arguments, control blocks, and the device-side synchronisation primitives
// (grid barrier, bounded doorbell waits) every persistent stage worker uses.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/camelot.h"

namespace camelot {

constexpr int kThreads = 256;          // 4 wave64s per workgroup
constexpr int kWaves = kThreads / 64;
// Worker grid = one workgroup per CU of the share. The dispatcher spreads a grid's
// workgroups evenly over the shader engines of each XCD whatever the number of CUs
// each engine has in the mask, so a CU can receive up to twice the average; every
// stage kernel fits at least 2 workgroups per CU, which keeps the grid co-resident.
constexpr int kWgPerCu = 1;
constexpr int kMinWgPerCuResident = 2;  // residency a worker kernel must allow (dispatch slack)
constexpr int kMaxRegsResident = 512 / kMinWgPerCuResident;          // registers per lane
constexpr size_t kMaxLdsResident = 160 * 1024 / kMinWgPerCuResident; // LDS bytes per workgroup
constexpr int kMaxBatch = CAMELOT_MAX_BATCH;
constexpr int kMaxStages = CAMELOT_MAX_STAGES;
constexpr int kMaxWorkers = CAMELOT_MAX_WORKERS;    // stage instances of one pipeline
constexpr int kSlotHeaderBytes = 4096;

// Status codes a worker reports (0 = ok / running).
enum WorkerStatus : int32_t {
  kStatusOk = 0,
  kStatusIdleExit = 1,     // idle longer than the idle timeout: exited cleanly
  kStatusTimeout = 2,      // a bounded wait inside a batch expired
  kStatusAborted = 3,      // another worker of the same grid aborted
  kStatusStopped = 4,      // host asked to stop
};

// Header at the start of every ring slot (device memory). Written by the producer
// stage's control workgroup before the slot's doorbell is rung.
struct SlotHeader {
  uint64_t seq;
  uint32_t n_req;
  uint32_t n_rows;
  uint64_t t_stage[2 * kMaxStages];     // device ticks: start/end of each stage so far
  uint64_t req_id[kMaxBatch];
  uint64_t req_tarr[kMaxBatch];         // arrival, device ticks
  uint32_t req_rows[kMaxBatch];
};
static_assert(sizeof(SlotHeader) <= kSlotHeaderBytes, "slot header too large");

// One request of the ingest table (replay: device memory; host: pinned ring).
struct IngestRec {
  uint64_t id;
  uint64_t t_arr;          // device ticks (absolute)
  uint64_t payload_off;    // byte offset of the request's first row in the payload base
  uint32_t rows;
  uint32_t valid;          // host ring: == lap+1 once written (torn-read guard)
};

// Result record header in the egress ring (pinned host memory), followed by
// k int32 indices and k f32 values.
struct EgressRec {
  uint64_t id;
  uint32_t row;
  uint32_t n_out;
  uint64_t t_arr;
  uint64_t t_done;
  uint64_t t_stage[2 * kMaxStages];
  // egress position + 1, written by the wave that wrote the record once its other
  // stores are acknowledged: the host takes a record only when this word matches
  // (the published egress head alone does not order the stores of other CUs
  // against it on their way to host memory)
  uint64_t seq;
};

// Host-written, device-read control block (pinned).
struct HostCtl {
  uint64_t stop;
  uint64_t pad0[15];
  uint64_t ingest_head;    // requests published by the host
  uint64_t pad1[15];
  uint64_t egress_tail;    // result rows consumed by the host
  uint64_t pad2[15];
};

// Device-written, host-read block (pinned). One writer per field.
struct DevPub {
  uint64_t t0;                              // epoch (device ticks)
  uint64_t egress_head;                     // result rows published
  uint64_t ingest_tail;                     // requests taken by stage 0
  uint64_t batches[kMaxWorkers];   // per worker (stage instance) below
  uint64_t id_sum[kMaxWorkers];
  uint64_t id_xor[kMaxWorkers];
  uint64_t rows[kMaxWorkers];               // rows finished
  uint64_t busy_ticks[kMaxWorkers];          // sum over batches of (publish - batch start)
  uint64_t wait_ticks[kMaxWorkers];          // sum of the waits for input and output space
  int32_t status[kMaxWorkers];
  int32_t started[kMaxWorkers];
  uint64_t pad[16];
};

// One batch's descriptor, written by the control workgroup before its broadcast.
struct BatchDesc {
  uint32_t stop;                  // nonzero: the workers exit with this status
  uint32_t rows;
  uint8_t* out;                   // payload of the output slot (ring output)
  SlotHeader* out_hdr;            // header of the output slot (ring output)
  uint64_t egress_base;           // egress row index of this batch's first row
  uint64_t t_stage[2 * kMaxStages];   // stage timestamps of the batch so far
  const uint8_t* rowptr[kMaxBatch];   // input row pointers
  const uint8_t* rowside[kMaxBatch];  // input side bytes of each row (side_bytes > 0)
  uint64_t row_id[kMaxBatch];         // (request id) per row
  uint32_t row_idx[kMaxBatch];        // row index within its request
  uint64_t row_tarr[kMaxBatch];
};

// Per-worker device control block (device memory, zeroed at creation).
struct WorkerCtl {
  // hierarchical grid barrier: workgroup g arrives on group counter g % 8, the last
  // arrival of each group on the top counter; release words per group
  uint32_t bar_group[8][32];      // one 128-byte line per group
  uint32_t bar_top;    uint32_t pad0[31];
  uint32_t bar_gen[8][32];        // release generation, one line per group
  uint32_t abort;      uint32_t pad2[31];
  uint32_t diag_arrived, diag_nwg, diag_group;   // filled on a barrier timeout
  uint32_t diag_pad;
  // batch descriptors, double-buffered by the batch's number in the launch (the
  // control workgroup writes the next batch's while the current one runs)
  BatchDesc dd[2];
  // persistent state
  uint64_t next_seq;              // next batch sequence number
  uint64_t ingest_cursor;         // stage 0: next request to take
  uint64_t egress_head;            // result rows written (terminal stage)
  uint64_t egress_tail_seen;       // the host's egress tail as last read (it only grows)
  uint64_t ticks_bench;           // bench mode: elapsed device ticks
  uint64_t reps_bench;            // bench mode: batches run
  uint32_t bench_stop[2];         // bench mode: workgroup 0's decision to stop, by rep parity
  uint64_t sum_acc, xor_acc, batches_acc;
  uint64_t rows_acc, busy_acc, wait_acc;
  // the control workgroup's batch broadcast (seq + 1), one 128-byte line per group so
  // that the idle workgroups' polls spread over 8 lines instead of one
  alignas(128) uint32_t go[8][32];
  // per group of compute workgroups (index mod 8): batches finished, summed over the
  // group's workgroups (cumulative; the control workgroup waits on these)
  alignas(128) uint32_t done[8][32];
};

// Stage parameters (device pointers borrowed from the caller or owned by the
// library's stage object).
struct StageParams {
  int32_t kind;
  int32_t n_layers;
  int32_t dims[CAMELOT_MAX_LAYERS + 1];
  int32_t k;
  int32_t in_row_bytes;
  int32_t out_row_bytes;
  const void* w[CAMELOT_MAX_LAYERS];
  uint16_t* scratch;              // MLP: two [kMaxBatch][max_dim] BF16 buffers
  int32_t scratch_stride;         // elements per scratch row
  const float* tables;            // LOGMEL: window, twiddles, mel filters
  float* partial;                 // CONV_POOL: per-tile channel sums [kMaxBatch][tiles][Cout]
};

enum InKind : int32_t { kInRing = 0, kInReplay = 1, kInHost = 2, kInBench = 3 };
enum OutKind : int32_t { kOutRing = 0, kOutEgress = 1, kOutBench = 2 };

struct WorkerArgs {
  StageParams sp;
  int32_t stage_index;
  int32_t n_stages;
  int32_t worker_index;           // slot of this stage instance in the published counters
  int32_t n_inst;                 // instances of this stage: this one takes every n_inst-th batch
  int32_t ctl_wg;                 // 1: one more workgroup, the last, only controls (persistent worker)
  int32_t max_batch;
  int32_t side_bytes;             // per-row bytes carried through the stages
  int32_t in_row_stride;          // stage 0: bytes between payload rows (row + side)
  int64_t in_side_off;            // ring input: offset of the side plane in a slot
  int64_t out_side_off;           // ring output: same for the output slot
  int32_t batch_target;
  int64_t batch_timeout_ticks;
  int64_t idle_ticks;             // exit after this long with nothing to do
  int64_t spin_ticks;             // limit of any wait inside a batch
  // input
  int32_t in_kind;
  int32_t in_depth;
  uint8_t* in_ring;               // ring base (slot i at in_ring + i * in_stride)
  uint64_t* in_state;             // per-slot state words
  int32_t in_state_sys;           // state words live in pinned host memory
  int64_t in_stride;
  const IngestRec* ingest;        // replay table or host ring
  int64_t n_ingest;               // replay: count; host: ring capacity
  const uint8_t* ingest_payload;  // payload base
  // output
  int32_t out_kind;
  int32_t out_depth;
  uint8_t* out_ring;
  uint64_t* out_state;
  int32_t out_state_sys;
  int64_t out_stride;
  uint8_t* egress;                // pinned host ring of records
  int64_t egress_cap;
  int32_t rec_bytes;
  // control
  WorkerCtl* ctl;
  HostCtl* hctl;
  DevPub* pub;
  // bench mode
  const uint8_t* bench_in;
  uint8_t* bench_out;
  int32_t bench_rows;
  int32_t bench_reps;             // upper bound on batches
  int64_t bench_ticks;            // > 0: stop after this much device time
};

// Handoff benchmark arguments (handoff.hip).
struct HandoffArgs {
  uint8_t* ring;            // depth * slot_bytes
  uint32_t* full;           // [depth][nwg] : times the chunk was filled
  uint32_t* freed;          // [depth][nwg] : times the chunk was consumed
  int64_t slot_bytes;
  int32_t depth;
  int64_t n_slots;
  int64_t chunk_bytes;      // multiple of 16
  int64_t spin_ticks;
  uint64_t* result;         // [0] sum, [1] xor, [2] t_first (min), [3] t_last (max), [4] error
};

#if defined(__HIP_DEVICE_COMPILE__) || defined(__HIPCC__)

// ---------------------------------------------------------------- device helpers
__device__ __forceinline__ uint64_t now_ticks() { return (uint64_t)wall_clock64(); }

template <typename T>
__device__ __forceinline__ T ld_acquire_agent(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_release_agent(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T ld_acquire_sys(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
}
template <typename T>
__device__ __forceinline__ void st_release_sys(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}
template <typename T>
__device__ __forceinline__ void st_relaxed_sys(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// SplitMix64 output function on id + golden gamma (first output for seed = id).
__device__ __host__ __forceinline__ uint64_t id_hash(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Grid-wide barrier for a persistent grid of nwg co-resident workgroups.
// Two levels: workgroups arrive on one of 8 group counters (group = block index
// mod 8, the XCD a workgroup lands on under round-robin dispatch), the last
// arrival of a group arrives on the top counter, and the last group releases every
// group's generation word. Memory ordering costs one agent-scope release fence
// (L2 write-back) and one acquire fence (invalidate) per workgroup, issued by
// thread 0 after the workgroup barrier has made every wave's stores complete;
// polling uses relaxed loads. Counter resets are waited on (s_waitcnt) before the
// next arrival can depend on them. The wait is bounded: on expiry, or when another
// workgroup aborted, returns false (and sets ctl->abort).
// Workgroup barrier before one thread publishes the workgroup's stores with a flag.
// Every wave releases its own stores at agent scope first (an L2 write-back per wave):
// thread 0's write-back alone after the barrier did not always cover the other
// waves' stores on gfx950 (a reader on another XCD then saw old data behind a new
// flag).
__device__ __forceinline__ void wg_barrier_stores_done() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
}

// Pause between two polls of a flag other workgroups will write: short naps while
// the flag is expected soon, longer ones once the wait is long (an idle worker),
// so idle pollers do not keep a memory channel busy.
__device__ __forceinline__ void poll_backoff(uint32_t polls) {
  if (polls < 64) __builtin_amdgcn_s_sleep(1);
  else if (polls < 1024) __builtin_amdgcn_s_sleep(4);
  else __builtin_amdgcn_s_sleep(32);
}


// The barrier in two halves: arrive publishes this workgroup's writes and counts
// it in; wait returns once every workgroup has arrived. Work that reads nothing
// the other workgroups write (loading constant weights) may run in between.
// sys_release: publish the workgroup's writes at system scope (results written to
// pinned host memory, or slots a DMA copy reads) instead of agent scope.
struct BarTicket {
  uint32_t gen;    // generation word seen at arrival (thread 0)
  bool wait;       // false for the workgroup that released the barrier
};

// wgi: this workgroup's index among the nwg that take part (default: blockIdx.x).
// wave_release = false: the caller's cross-workgroup stores were written through
// (cache policy sc1), so thread 0's release alone publishes them.
__device__ __forceinline__ BarTicket grid_arrive(WorkerCtl* ctl, uint32_t nwg, bool sys_release = false,
                                                 int wgi = -1, bool wave_release = true) {
  BarTicket t{0u, false};
  if (wave_release) {
    wg_barrier_stores_done();
  } else {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const uint32_t g = (wgi < 0 ? blockIdx.x : (uint32_t)wgi) & 7u;
    const uint32_t ngroups = nwg < 8u ? nwg : 8u;
    const uint32_t members = (nwg - g + 7u) >> 3;
    uint32_t* genp = &ctl->bar_gen[g][0];
    if (sys_release) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
    else __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    t.gen = __hip_atomic_load(genp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    t.wait = true;
    const uint32_t prev = __hip_atomic_fetch_add(&ctl->bar_group[g][0], 1u, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
    if (prev == members - 1) {
      __hip_atomic_store(&ctl->bar_group[g][0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_s_waitcnt(0);
      const uint32_t top = __hip_atomic_fetch_add(&ctl->bar_top, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (top == ngroups - 1) {
        __hip_atomic_store(&ctl->bar_top, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
        for (uint32_t q = 0; q < ngroups; ++q)
          __hip_atomic_store(&ctl->bar_gen[q][0], t.gen + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        t.wait = false;
      }
    }
  }
  return t;
}

__device__ __forceinline__ bool grid_wait(WorkerCtl* ctl, uint32_t nwg, BarTicket t, int64_t spin_ticks,
                                          int wgi = -1) {
  __shared__ int s_ok;
  if (threadIdx.x == 0) {
    int ok = 1;
    const uint32_t g = (wgi < 0 ? blockIdx.x : (uint32_t)wgi) & 7u;
    uint32_t* genp = &ctl->bar_gen[g][0];
    if (t.wait) {
      const uint64_t t0 = now_ticks();
      uint32_t polls = 0;
      while (__hip_atomic_load(genp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == t.gen) {
        ++polls;
        if ((polls & 15u) == 0 && __hip_atomic_load(&ctl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          ok = 0;
          break;
        }
        if ((int64_t)(now_ticks() - t0) > spin_ticks) {
          // record who was missing: arrivals on this group and on the top counter
          ctl->diag_arrived = __hip_atomic_load(&ctl->bar_group[g][0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) |
                              (__hip_atomic_load(&ctl->bar_top, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) << 16);
          ctl->diag_nwg = nwg;
          ctl->diag_group = g;
          __hip_atomic_store(&ctl->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
        poll_backoff(polls);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

__device__ __forceinline__ bool grid_barrier(WorkerCtl* ctl, uint32_t nwg, int64_t spin_ticks,
                                             bool sys_release = false, int wgi = -1, bool wave_release = true) {
  return grid_wait(ctl, nwg, grid_arrive(ctl, nwg, sys_release, wgi, wave_release), spin_ticks, wgi);
}

// Intra-wave LDS hand-off: orders this wave's LDS writes before its later reads
// by other lanes of the same wave.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

#endif  // device

}  // namespace camelot
