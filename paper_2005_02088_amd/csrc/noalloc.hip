// camelot_stage_run_noalloc: the one-shot stage run of camelot_stage_run without any
// device allocation, for callers that cannot allocate (code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc).
//
// Everything camelot_stage_run allocates per call lives here in one file-scope
// device array instead: the worker's control block (grid-barrier counters, batch
// descriptors), the log-mel tables and the stage's scratch (the MLP's hidden state,
// the convolution's per-tile partial sums). Each device holds its own copy of the
// array until the process ends; host code reaches it only through the address
// hipGetSymbolAddress returns for the current device, never through its name.
// Calls on one device share that copy: two calls whose work overlaps on the device
// race on it.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "internal.h"

namespace camelot {
namespace {

constexpr int64_t kStageScratchMax = CAMELOT_NOALLOC_SCRATCH_BYTES;
constexpr int64_t kCtlBytes = ((int64_t)sizeof(WorkerCtl) + 255) / 256 * 256;
constexpr int64_t kTabBytes = ((int64_t)kLogmelTableFloats * 4 + 255) / 256 * 256;
constexpr int64_t kScratchBytes = kCtlBytes + kTabBytes + kStageScratchMax;
constexpr int kMaxDevices = 64;

// [control block | log-mel tables | stage scratch]
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

// Clears the control block (the barrier counters and descriptors must start at zero).
__global__ void __launch_bounds__(256) zero_words(uint32_t* p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

// Writes one chunk of the log-mel tables, carried in the kernel's arguments (no host
// buffer, no copy node: the launch alone moves the values, also under capture).
constexpr int kTabChunk = 576;
static_assert(kLogmelTableFloats % kTabChunk == 0, "table chunks must tile the table");
struct TabChunk {
  float v[kTabChunk];
};
__global__ void __launch_bounds__(256) put_table_chunk(float* dst, TabChunk c) {
  for (int i = threadIdx.x; i < kTabChunk; i += blockDim.x) dst[i] = c.v[i];
}

std::mutex g_mu;
uint8_t* g_base[kMaxDevices] = {nullptr};   // the array's device address, per device
bool g_tables_ready[kMaxDevices] = {false};

// The array's address on the current device (looked up once per device).
int32_t scratch_base(int dev, uint8_t** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_base[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(CAMELOT_EDEVICE, "hipGetSymbolAddress of the scratch array on device %d: %s", dev,
                  hipGetErrorString(e));
    g_base[dev] = (uint8_t*)p;
  }
  *out = g_base[dev];
  return CAMELOT_OK;
}

int32_t put_tables(float* dst, hipStream_t s) {
  float t[kLogmelTableFloats];
  if (!logmel_tables(t)) return fail(CAMELOT_EINVAL, "log-mel tables exceed the kernel's LDS table");
  for (int c = 0; c < kLogmelTableFloats / kTabChunk; ++c) {
    TabChunk ch;
    std::memcpy(ch.v, t + c * kTabChunk, sizeof ch.v);
    put_table_chunk<<<1, 256, 0, s>>>(dst + c * kTabChunk, ch);
    HIP_TRY(hipGetLastError());
  }
  return CAMELOT_OK;
}

}  // namespace
}  // namespace camelot

using namespace camelot;

extern "C" int32_t camelot_stage_run_noalloc(const camelot_stage_desc* stage, const void* in, void* out,
                                             int32_t rows, int32_t n_cus, int32_t reps, void* stream) {
  clear_error();
  // every argument is checked on the host before the device is touched
  StageParams sp;
  int64_t sb = 0;
  int32_t rc = stage_params(stage, &sp, &sb);
  if (rc) return rc;
  if (sb > kStageScratchMax)
    return fail(CAMELOT_EINVAL,
                "stage kind %d needs %lld scratch bytes; the allocation-free run holds at most %lld "
                "(use camelot_stage_run)",
                stage->kind, (long long)sb, (long long)kStageScratchMax);
  if (n_cus < 8 || n_cus % 8 != 0 || n_cus > 256)
    return fail(CAMELOT_EINVAL, "n_cus must be a multiple of 8 in 8..256 (got %d)", n_cus);
  if (rows < 0 || rows > kMaxBatch) return fail(CAMELOT_EINVAL, "rows must be in 0..%d", kMaxBatch);
  if (reps < 1) return fail(CAMELOT_EINVAL, "reps must be >= 1");
  if (rows > 0 && (!in || !out)) return fail(CAMELOT_EINVAL, "in/out are NULL");

  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(CAMELOT_EINVAL, "device %d beyond %d", dev, kMaxDevices);
  int dev_cus = 0, wclk_khz = 0;
  HIP_TRY(hipDeviceGetAttribute(&dev_cus, hipDeviceAttributeMultiprocessorCount, dev));
  HIP_TRY(hipDeviceGetAttribute(&wclk_khz, hipDeviceAttributeWallClockRate, dev));
  if (n_cus > dev_cus) return fail(CAMELOT_EINVAL, "n_cus %d exceeds the device's %d CUs", n_cus, dev_cus);
  uint8_t* base = nullptr;
  if ((rc = scratch_base(dev, &base))) return rc;
  WorkerCtl* ctl = (WorkerCtl*)base;
  float* tab = (float*)(base + kCtlBytes);
  uint8_t* stage_scratch = base + kCtlBytes + kTabBytes;

  hipStream_t s = (hipStream_t)stream;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  HIP_TRY(hipStreamIsCapturing(s, &cap));
  if (stage->kind == CAMELOT_STAGE_LOGMEL) {
    bool ready;
    {
      std::lock_guard<std::mutex> lk(g_mu);
      ready = g_tables_ready[dev];
    }
    // Outside capture the tables are written once per device and the stream waited
    // for; a captured call records their writes in the graph every time, since the
    // graph may run before any eager call has written them.
    if (!ready || cap != hipStreamCaptureStatusNone) {
      if ((rc = put_tables(tab, s))) return rc;
      if (cap == hipStreamCaptureStatusNone) {
        HIP_TRY(hipStreamSynchronize(s));
        std::lock_guard<std::mutex> lk(g_mu);
        g_tables_ready[dev] = true;
      }
    }
  }
  stage_params_bind(&sp, sb > 0 ? stage_scratch : nullptr, tab);

  // the control block starts at zero for every run (a fill kernel, not a memset node)
  zero_words<<<8, 256, 0, s>>>((uint32_t*)ctl, (int)(sizeof(WorkerCtl) / 4));
  HIP_TRY(hipGetLastError());

  WorkerArgs a;
  std::memset(&a, 0, sizeof a);
  a.sp = sp;
  a.stage_index = 0;
  a.n_stages = 1;
  a.max_batch = kMaxBatch;
  a.spin_ticks = 2LL * wclk_khz * 1000;   // 2 s limit on any in-batch wait
  a.idle_ticks = a.spin_ticks;
  a.in_kind = kInBench;
  a.out_kind = is_result_stage(stage->kind) ? kOutBench : kOutRing;
  a.ctl = ctl;
  a.bench_in = (const uint8_t*)in;
  a.bench_out = (uint8_t*)out;
  a.bench_rows = rows;
  a.bench_reps = reps;
  a.side_bytes = (int32_t)stage_side_bytes(stage);
  a.in_row_stride = a.sp.in_row_bytes + a.side_bytes;
  return launch_worker(stage->kind, a, n_cus, s);
}
