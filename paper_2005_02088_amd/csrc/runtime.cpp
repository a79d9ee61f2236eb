// Host side of libcamelot: device query, stage objects, CU-masked streams, the
// pipeline (rings, doorbells, ingest/egress, persistent workers, host-staged relay
// for the baseline), the handoff benchmark and the predictor entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/camelot.h"
#include "device_common.h"
#include "errors.h"
#include "internal.h"

namespace camelot {

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;

int32_t fail(int32_t code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}
void clear_error() { g_err.clear(); }


const void* worker_kernel(int kind, bool bench);   // stages.hip

// All library allocations, fills and frees go through one non-blocking stream with
// stream-ordered allocation: the CU-masked streams of live pipelines are blocking
// streams that hold persistent workers, and anything that synchronises with them
// (null-stream copies, hipFree, hipDeviceSynchronize) would wait for those workers.
static hipStream_t g_mem_stream = nullptr;
static std::mutex g_mem_mu;
hipStream_t mem_stream() {
  std::lock_guard<std::mutex> lk(g_mem_mu);
  if (!g_mem_stream) (void)hipStreamCreateWithFlags(&g_mem_stream, hipStreamNonBlocking);
  return g_mem_stream;
}
int32_t dmalloc(void** ptr, size_t bytes) {
  hipStream_t s = mem_stream();
  HIP_TRY(hipMallocAsync(ptr, bytes, s));
  HIP_TRY(hipStreamSynchronize(s));
  return CAMELOT_OK;
}
void dfree(void* ptr) {
  if (ptr) (void)hipFreeAsync(ptr, mem_stream());
}
int32_t dzero(void* ptr, size_t bytes) {
  hipStream_t s = mem_stream();
  HIP_TRY(hipMemsetAsync(ptr, 0, bytes, s));
  HIP_TRY(hipStreamSynchronize(s));
  return CAMELOT_OK;
}
int32_t d2h(void* dst, const void* src, size_t bytes) {
  hipStream_t s = mem_stream();
  HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return CAMELOT_OK;
}
int32_t h2d(void* dst, const void* src, size_t bytes) {
  hipStream_t s = mem_stream();
  HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  return CAMELOT_OK;
}

extern "C" __global__ void camelot_handoff_producer(HandoffArgs);
extern "C" __global__ void camelot_handoff_consumer(HandoffArgs);

// ------------------------------------------------------------------ device info
static std::mutex g_mu;
static DevInfo g_dev;

int32_t dev_info(DevInfo* out) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_dev.ok) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    hipDeviceProp_t p;
    HIP_TRY(hipGetDeviceProperties(&p, dev));
    int wclk = 0;
    HIP_TRY(hipDeviceGetAttribute(&wclk, hipDeviceAttributeWallClockRate, dev));
    g_dev.n_cus = p.multiProcessorCount;
    g_dev.wclk_hz = (int64_t)wclk * 1000;
    g_dev.mem = (int64_t)p.totalGlobalMem;
    std::snprintf(g_dev.arch, sizeof g_dev.arch, "%s", p.gcnArchName);
    g_dev.ok = true;
  }
  *out = g_dev;
  return CAMELOT_OK;
}

int64_t ns_to_ticks(int64_t ns, int64_t hz) { return (int64_t)((long double)ns * hz / 1e9L); }
static uint64_t ticks_to_ns(int64_t ticks, int64_t hz) {
  return ticks <= 0 ? 0 : (uint64_t)((long double)ticks * 1e9L / hz);
}
static int64_t host_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------------ CU masks & streams
// Logical CU-mask bits are dealt round-robin over the XCDs by the driver, so a
// contiguous range of a multiple of 8 bits gives the same number of CUs on every XCD.
static void build_mask(int offset, int n, uint32_t mask[8]) {
  std::memset(mask, 0, 8 * sizeof(uint32_t));
  for (int b = offset; b < offset + n && b < 256; ++b) mask[b / 32] |= 1u << (b % 32);
}

static int32_t make_masked_stream(int offset, int n, hipStream_t* s) {
  uint32_t mask[8];
  build_mask(offset, n, mask);
  HIP_TRY(hipExtStreamCreateWithCUMask(s, 8, mask));
  return CAMELOT_OK;
}

// Cache of masked streams used by the one-shot stage runs (profiling, co-location
// runs, the handoff benchmark). Every CU-masked stream holds a hardware queue of its
// own, and a process that holds more queues than the device has queue slots gets
// them time-sliced, which stalls persistent workers (measured: the MLP stage at
// batch 128 on 136 CUs took 94 us with up to 16 extra idle masked streams alive,
// 113 us with 32 and 217 us with 48). So the cache is small: past
// kMaxCachedStreams the least recently used stream is drained and destroyed.
// The calls that use these streams synchronize them before returning, so an
// evicted stream is idle (they are not meant to run concurrently from several
// host threads).
constexpr size_t kMaxCachedStreams = 4;
struct CachedStream {
  hipStream_t s;
  uint64_t last_use;
};
static std::map<std::pair<int, int>, CachedStream> g_streams;
static uint64_t g_stream_clock = 0;
int32_t new_masked_stream(int offset, int n, hipStream_t* s) { return make_masked_stream(offset, n, s); }

// Drops the cached streams (all idle): a pipeline's persistent workers then share
// the device's hardware queues with as few other queues as possible.
static void release_cached_streams() {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& kv : g_streams) {
    (void)hipStreamSynchronize(kv.second.s);
    (void)hipStreamDestroy(kv.second.s);
  }
  g_streams.clear();
}

int32_t cached_stream(int offset, int n, hipStream_t* s) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_streams.find({offset, n});
  if (it != g_streams.end()) {
    it->second.last_use = ++g_stream_clock;
    *s = it->second.s;
    return CAMELOT_OK;
  }
  if (g_streams.size() >= kMaxCachedStreams) {
    auto lru = g_streams.begin();
    for (auto jt = g_streams.begin(); jt != g_streams.end(); ++jt)
      if (jt->second.last_use < lru->second.last_use) lru = jt;
    (void)hipStreamSynchronize(lru->second.s);
    (void)hipStreamDestroy(lru->second.s);
    g_streams.erase(lru);
  }
  int32_t rc = make_masked_stream(offset, n, s);
  if (rc) return rc;
  g_streams[{offset, n}] = CachedStream{*s, ++g_stream_clock};
  return CAMELOT_OK;
}

// ------------------------------------------------------------------ log-mel tables
// Window, FFT twiddles and the HTK mel filterbank (40 triangles on 42 points equally
// spaced in mel over 0..8 kHz, evaluated at the bin frequencies k * 16000 / 512),
// computed in double and stored as float.
bool logmel_tables(float* t) {
  const double PI = 3.14159265358979323846;
  std::fill(t, t + kLogmelTableFloats, 0.f);
  for (int n = 0; n < 400; ++n) t[n] = (float)(0.54 - 0.46 * std::cos(2 * PI * n / 399.0));
  for (int q = 0; q < 256; ++q) {
    t[400 + 2 * q] = (float)std::cos(-2 * PI * q / 256.0);
    t[400 + 2 * q + 1] = (float)std::sin(-2 * PI * q / 256.0);
  }
  for (int k = 0; k <= 256; ++k) {
    t[912 + 2 * k] = (float)std::cos(-2 * PI * k / 512.0);
    t[912 + 2 * k + 1] = (float)std::sin(-2 * PI * k / 512.0);
  }
  auto mel = [](double f) { return 2595.0 * std::log10(1.0 + f / 700.0); };
  auto hz = [](double m) { return 700.0 * (std::pow(10.0, m / 2595.0) - 1.0); };
  double pts[42];
  const double top = mel(8000.0);
  for (int i = 0; i < 42; ++i) pts[i] = hz(top * i / 41.0);
  // per band: first bin, bin count, offset of its weights; the weights follow at 1546
  int nw = 0;
  for (int m = 0; m < 40; ++m) {
    const double lo = pts[m], c = pts[m + 1], hi = pts[m + 2];
    int first = -1, last = -1;
    double wk[257];
    for (int k = 0; k <= 256; ++k) {
      const double f = k * 16000.0 / 512.0;
      double v = 0.0;
      if (f >= lo && f <= c) v = (f - lo) / (c - lo);
      else if (f > c && f <= hi) v = (hi - f) / (hi - c);
      wk[k] = v;
      if (v > 0.0) { if (first < 0) first = k; last = k; }
    }
    if (first < 0) { first = 0; last = -1; }
    t[1426 + 3 * m] = (float)first;
    t[1426 + 3 * m + 1] = (float)(last - first + 1);
    t[1426 + 3 * m + 2] = (float)nw;
    for (int k = first; k <= last; ++k) {
      // cannot overflow for 40 bands over 257 bins; the caller reports it if it did
      if (1546 + nw >= kLogmelTableFloats) return false;
      t[1546 + nw++] = (float)wk[k];
    }
  }
  return true;
}

static float* g_logmel_dev = nullptr;
static int32_t logmel_device_tables(const float** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_logmel_dev) {
    std::vector<float> t(kLogmelTableFloats);
    if (!logmel_tables(t.data())) return fail(CAMELOT_EINVAL, "log-mel tables exceed the kernel's LDS table");
    float* d = nullptr;
    int32_t rc = dmalloc(&d, t.size() * sizeof(float));
    if (!rc) rc = h2d(d, t.data(), t.size() * sizeof(float));
    if (rc) return rc;
    g_logmel_dev = d;
  }
  *out = g_logmel_dev;
  return CAMELOT_OK;
}

// ------------------------------------------------------------------ stages
bool is_result_stage(int kind) {
  return kind == CAMELOT_STAGE_GEMM_ARGMAX || kind == CAMELOT_STAGE_TOPK;
}

static int32_t check_stage(const camelot_stage_desc* d, int64_t* in_b, int64_t* out_b) {
  if (!d) return fail(CAMELOT_EINVAL, "stage descriptor is NULL");
  switch (d->kind) {
    case CAMELOT_STAGE_GEMM_RELU:
      if (d->dims[0] < 1 || d->dims[0] > 1024 || d->dims[1] < 1)
        return fail(CAMELOT_EINVAL, "GEMM_RELU needs 1 <= in_dim <= 1024 and out_dim >= 1");
      if (!d->weights[0]) return fail(CAMELOT_EINVAL, "GEMM_RELU needs weights[0]");
      *in_b = 4LL * d->dims[0];
      *out_b = 4LL * d->dims[1];
      return CAMELOT_OK;
    case CAMELOT_STAGE_GEMM_ARGMAX:
      if (d->dims[0] < 1 || d->dims[1] < 1 || d->dims[1] > 16)
        return fail(CAMELOT_EINVAL, "GEMM_ARGMAX needs in_dim >= 1 and 1 <= out_dim <= 16");
      if (!d->weights[0]) return fail(CAMELOT_EINVAL, "GEMM_ARGMAX needs weights[0]");
      *in_b = 4LL * d->dims[0];
      *out_b = 8;
      return CAMELOT_OK;
    case CAMELOT_STAGE_LOGMEL:
      *in_b = 4LL * 2000;
      *out_b = 4LL * 440;
      return CAMELOT_OK;
    case CAMELOT_STAGE_MLP_BF16: {
      const int L = d->n_layers;
      if (L < 1 || L > CAMELOT_MAX_LAYERS) return fail(CAMELOT_EINVAL, "MLP_BF16 needs 1..%d layers", CAMELOT_MAX_LAYERS);
      for (int l = 0; l <= L; ++l) {
        if (d->dims[l] < 8 || d->dims[l] % 8 != 0) return fail(CAMELOT_EINVAL, "MLP_BF16 dims must be multiples of 8");
        if (l >= 1 && d->dims[l] % 16 != 0) return fail(CAMELOT_EINVAL, "MLP_BF16 layer widths must be multiples of 16");
        if (d->dims[l] > 16384) return fail(CAMELOT_EINVAL, "MLP_BF16 dims must be <= 16384");
      }
      for (int l = 0; l < L; ++l)
        if (!d->weights[l]) return fail(CAMELOT_EINVAL, "MLP_BF16 needs weights[%d]", l);
      *in_b = 4LL * d->dims[0];
      *out_b = 4LL * d->dims[L];
      return CAMELOT_OK;
    }
    case CAMELOT_STAGE_TOPK:
      if (d->dims[0] < 1 || d->dims[0] > 4096) return fail(CAMELOT_EINVAL, "TOPK needs 1 <= in_dim <= 4096");
      if (d->k < 1 || d->k > CAMELOT_MAX_K || d->k > d->dims[0])
        return fail(CAMELOT_EINVAL, "TOPK needs 1 <= k <= min(in_dim, %d)", CAMELOT_MAX_K);
      *in_b = 4LL * d->dims[0];
      *out_b = 8LL * d->k;
      return CAMELOT_OK;
    case CAMELOT_STAGE_GATHER:
      if (d->dims[0] < 1 || d->dims[0] > 4096) return fail(CAMELOT_EINVAL, "GATHER needs 1..4096 ids per row");
      if (d->dims[1] < 64 || d->dims[1] > 1024 || d->dims[1] % 64 != 0)
        return fail(CAMELOT_EINVAL, "GATHER needs dim in 64..1024, a multiple of 64");
      if (d->k < 1) return fail(CAMELOT_EINVAL, "GATHER needs the table row count in k");
      if (!d->weights[0]) return fail(CAMELOT_EINVAL, "GATHER needs weights[0] (the table)");
      *in_b = 4LL * d->dims[0];
      *out_b = 4LL * d->dims[1];
      return CAMELOT_OK;
    case CAMELOT_STAGE_CONV_POOL:
      if (d->dims[0] < 1 || d->dims[1] < 1 || d->dims[0] * d->dims[1] > (1 << 20) || d->dims[2] != 64 ||
          d->dims[3] != 64)
        return fail(CAMELOT_EINVAL, "CONV_POOL needs H, W >= 1 (H*W <= 2^20) and 64 input and output channels");
      if (!d->weights[0]) return fail(CAMELOT_EINVAL, "CONV_POOL needs weights[0]");
      *in_b = 2LL * d->dims[0] * d->dims[1] * d->dims[2];
      *out_b = 4LL * d->dims[3];
      return CAMELOT_OK;
    case CAMELOT_STAGE_GATHER_SCORE:
      if (d->dims[1] < 1 || d->dims[0] < d->dims[1] || d->dims[0] % d->dims[1] != 0 || d->dims[0] > 1024)
        return fail(CAMELOT_EINVAL, "GATHER_SCORE needs dims[0] = heads * dims[1] <= 1024");
      if (d->dims[2] < 1 || d->dims[2] > 1024) return fail(CAMELOT_EINVAL, "GATHER_SCORE needs 1..1024 ids");
      if (d->k < 1 || !d->weights[0]) return fail(CAMELOT_EINVAL, "GATHER_SCORE needs the table and its rows in k");
      *in_b = 4LL * d->dims[0];
      *out_b = 4LL * (d->dims[0] / d->dims[1]) * d->dims[2];
      return CAMELOT_OK;
    case CAMELOT_STAGE_ARTIFACT_P:
    case CAMELOT_STAGE_ARTIFACT_M:
      if (d->dims[0] < 1024 || d->dims[0] > 16384 || d->dims[0] % 1024 != 0)
        return fail(CAMELOT_EINVAL, "artifact stages need D = dims[0], a multiple of 1024 up to 16384");
      if (d->dims[1] < d->dims[0] || d->dims[1] % d->dims[0] != 0 || d->k < d->dims[1])
        return fail(CAMELOT_EINVAL, "ARTIFACT_P/M need dims[1] a multiple of D and a table of k >= dims[1] words");
      if (!d->weights[0]) return fail(CAMELOT_EINVAL, "ARTIFACT_P/M need the table in weights[0]");
      *in_b = 4LL * d->dims[0];
      *out_b = 4LL * d->dims[0];
      return CAMELOT_OK;
    case CAMELOT_STAGE_ARTIFACT_C:
      if (d->dims[0] < 1024 || d->dims[0] > 16384 || d->dims[0] % 1024 != 0)
        return fail(CAMELOT_EINVAL, "artifact stages need D = dims[0], a multiple of 1024 up to 16384");
      if (d->dims[1] < 0 || d->dims[1] > (1 << 20)) return fail(CAMELOT_EINVAL, "ARTIFACT_C needs 0..2^20 iterations");
      *in_b = 4LL * d->dims[0];
      *out_b = 4LL * d->dims[0];
      return CAMELOT_OK;
    default:
      return fail(CAMELOT_EINVAL, "unknown stage kind %d", d->kind);
  }
}

// side bytes a stage needs in a one-shot run (ids following each input row)
int64_t stage_side_bytes(const camelot_stage_desc* d) {
  return d->kind == CAMELOT_STAGE_GATHER_SCORE ? 4LL * d->dims[2] : 0;
}

static int result_k(const camelot_stage_desc* d) {
  return d->kind == CAMELOT_STAGE_TOPK ? d->k : 1;
}

static int64_t stage_scratch_bytes(const camelot_stage_desc* d, int* stride) {
  *stride = 0;
  if (d->kind == CAMELOT_STAGE_CONV_POOL) {
    const int64_t tiles = ((int64_t)d->dims[0] * d->dims[1] + 63) / 64;
    return (int64_t)kMaxBatch * tiles * d->dims[3] * 4;
  }
  if (d->kind != CAMELOT_STAGE_MLP_BF16) return 0;
  int mx = 0;
  for (int l = 0; l <= d->n_layers; ++l) mx = std::max(mx, d->dims[l]);
  mx = (mx + 31) & ~31;    // whole 32-wide chunks (the fragment layout of the row path)
  *stride = mx;
  return 2LL * kMaxBatch * mx * 2;
}

StageRes::~StageRes() { dfree(scratch); }

int32_t stage_params(const camelot_stage_desc* d, StageParams* sp, int64_t* scratch_bytes) {
  int64_t in_b = 0, out_b = 0;
  int32_t rc = check_stage(d, &in_b, &out_b);
  if (rc) return rc;
  std::memset(sp, 0, sizeof(*sp));
  sp->kind = d->kind;
  sp->n_layers = d->n_layers;
  std::memcpy(sp->dims, d->dims, sizeof(sp->dims));
  sp->k = d->k;
  sp->in_row_bytes = (int32_t)in_b;
  sp->out_row_bytes = (int32_t)out_b;
  for (int l = 0; l < CAMELOT_MAX_LAYERS; ++l) sp->w[l] = d->weights[l];
  int stride = 0;
  *scratch_bytes = stage_scratch_bytes(d, &stride);
  sp->scratch_stride = stride;
  return CAMELOT_OK;
}

void stage_params_bind(StageParams* sp, void* scratch, const float* logmel_tab) {
  sp->scratch = (uint16_t*)scratch;
  if (sp->kind == CAMELOT_STAGE_CONV_POOL) sp->partial = (float*)scratch;
  if (sp->kind == CAMELOT_STAGE_LOGMEL) sp->tables = logmel_tab;
}

int32_t fill_params(const camelot_stage_desc* d, StageRes* res, StageParams* sp) {
  int64_t sb = 0;
  int32_t rc = stage_params(d, sp, &sb);
  if (rc) return rc;
  if (sb > 0 && !res->scratch) {
    rc = dmalloc(&res->scratch, sb);
    if (rc) return rc;
    res->scratch_bytes = sb;
  }
  const float* tab = nullptr;
  if (d->kind == CAMELOT_STAGE_LOGMEL && (rc = logmel_device_tables(&tab))) return rc;
  stage_params_bind(sp, res->scratch, tab);
  return CAMELOT_OK;
}

int32_t check_share(int n_cus, int offset, int total) {
  if (n_cus < 8 || n_cus % 8 != 0 || offset < 0 || offset % 8 != 0 || offset + n_cus > total)
    return fail(CAMELOT_EINVAL, "CU share %d at offset %d: need multiples of 8 within %d CUs", n_cus,
                offset, total);
  return CAMELOT_OK;
}

int32_t launch_worker(int kind, const WorkerArgs& a, int n_cus, hipStream_t s) {
  const void* fn = worker_kernel(kind, a.in_kind == kInBench);
  if (!fn) return fail(CAMELOT_EINVAL, "no worker for stage kind %d", kind);
  // One workgroup per CU is launched, but the dispatcher may place two on one CU of
  // the share (it balances workgroups over shader engines, not over the masked
  // CUs): a kernel that fits only once per CU could leave a workgroup unplaced and
  // its grid barriers could never complete. Refuse such a kernel instead: two
  // workgroups of 4 wave64s fit on a CU when each wave needs at most 256 of the
  // SIMD's 512 registers per lane and each workgroup at most half of the LDS.
  // Nor may it need scratch: the runtime may start fewer waves than the grid when it
  // cannot back every wave's scratch at once, which leaves workgroups unplaced too.
  hipFuncAttributes fa;
  HIP_TRY(hipFuncGetAttributes(&fa, fn));
  if (fa.numRegs > kMaxRegsResident || fa.sharedSizeBytes > kMaxLdsResident)
    return fail(CAMELOT_EDEVICE, "stage kind %d: %d registers and %zu LDS bytes per workgroup leave fewer than %d "
                "workgroups per CU", kind, fa.numRegs, (size_t)fa.sharedSizeBytes, kMinWgPerCuResident);
  if (fa.localSizeBytes > 0)
    return fail(CAMELOT_EDEVICE, "stage kind %d needs %zu bytes of scratch per lane; a worker grid must not",
                kind, (size_t)fa.localSizeBytes);
  void* args[] = {(void*)&a};
  // a persistent worker adds its control workgroup last: it shares a CU with one of
  // the compute workgroups, which are placed first, one per CU
  HIP_TRY(hipLaunchKernel(fn, dim3(kWgPerCu * n_cus + a.ctl_wg), dim3(kThreads), args, 0, s));
  return CAMELOT_OK;
}

}  // namespace camelot

using namespace camelot;

extern "C" int32_t camelot_stage_kernel_info(int32_t kind, int32_t one_shot, int32_t* regs, int64_t* lds_bytes,
                                             int32_t* fits) {
  clear_error();
  if (!regs || !lds_bytes || !fits) return fail(CAMELOT_EINVAL, "NULL output");
  const void* fn = worker_kernel(kind, one_shot != 0);
  if (!fn) return fail(CAMELOT_EINVAL, "no kernel for stage kind %d", kind);
  hipFuncAttributes fa;
  HIP_TRY(hipFuncGetAttributes(&fa, fn));
  *regs = fa.numRegs;
  *lds_bytes = (int64_t)fa.sharedSizeBytes;
  *fits = (fa.numRegs <= kMaxRegsResident && fa.sharedSizeBytes <= kMaxLdsResident && fa.localSizeBytes == 0) ? 1 : 0;
  return CAMELOT_OK;
}

// ==================================================================== C ABI
extern "C" const char* camelot_last_error(void) { return g_err.c_str(); }
extern "C" int32_t camelot_version(void) { return 100; }

extern "C" int32_t camelot_device_query(camelot_device_info* out) {
  clear_error();
  if (!out) return fail(CAMELOT_EINVAL, "out is NULL");
  DevInfo d;
  int32_t rc = dev_info(&d);
  if (rc) return rc;
  std::memset(out, 0, sizeof(*out));
  out->n_cus = d.n_cus;
  out->n_xcds = 8;
  out->wall_clock_hz = d.wclk_hz;
  out->hbm_bytes = d.mem;
  std::snprintf(out->arch, sizeof out->arch, "%s", d.arch);
  return CAMELOT_OK;
}

extern "C" int64_t camelot_stage_row_bytes_in(const camelot_stage_desc* stage) {
  clear_error();
  int64_t i = 0, o = 0;
  int32_t rc = check_stage(stage, &i, &o);
  return rc ? rc : i;
}

extern "C" int64_t camelot_stage_row_bytes_out(const camelot_stage_desc* stage) {
  clear_error();
  int64_t i = 0, o = 0;
  int32_t rc = check_stage(stage, &i, &o);
  return rc ? rc : o;
}

extern "C" int32_t camelot_stage_run(const camelot_stage_desc* stage, const void* in, void* out, int32_t rows,
                                     int32_t n_cus, int32_t cu_offset, int32_t reps, double* ns_per_rep,
                                     double* device_ns_per_rep) {
  clear_error();
  DevInfo dev;
  int32_t rc = dev_info(&dev);
  if (rc) return rc;
  if (n_cus == 0) { n_cus = dev.n_cus; cu_offset = 0; }
  if ((rc = check_share(n_cus, cu_offset, dev.n_cus))) return rc;
  if (rows < 0 || rows > kMaxBatch) return fail(CAMELOT_EINVAL, "rows must be in 0..%d", kMaxBatch);
  if (reps < 1) return fail(CAMELOT_EINVAL, "reps must be >= 1");
  if (rows > 0 && (!in || !out)) return fail(CAMELOT_EINVAL, "in/out are NULL");
  StageRes res;
  WorkerArgs a;
  std::memset(&a, 0, sizeof a);
  if ((rc = fill_params(stage, &res, &a.sp))) return rc;
  hipStream_t s;
  if ((rc = cached_stream(cu_offset, n_cus, &s))) return rc;
  WorkerCtl* ctl = nullptr;
  if ((rc = dmalloc(&ctl, sizeof(WorkerCtl)))) return rc;
  std::unique_ptr<WorkerCtl, void (*)(WorkerCtl*)> guard(ctl, [](WorkerCtl* p) { dfree(p); });
  if ((rc = dzero(ctl, sizeof(WorkerCtl)))) return rc;
  a.stage_index = 0;
  a.n_stages = 1;
  a.max_batch = kMaxBatch;
  a.spin_ticks = 2 * dev.wclk_hz;   // 2 s limit on any in-batch wait
  a.idle_ticks = 2 * dev.wclk_hz;
  a.in_kind = kInBench;
  a.out_kind = is_result_stage(stage->kind) ? kOutBench : kOutRing;
  a.ctl = ctl;
  a.bench_in = (const uint8_t*)in;
  a.bench_out = (uint8_t*)out;
  a.bench_rows = rows;
  a.bench_reps = reps;
  a.side_bytes = (int32_t)stage_side_bytes(stage);
  a.in_row_stride = a.sp.in_row_bytes + a.side_bytes;
  hipEvent_t ev0, ev1;
  HIP_TRY(hipEventCreate(&ev0));
  HIP_TRY(hipEventCreate(&ev1));
  HIP_TRY(hipEventRecord(ev0, s));
  rc = launch_worker(stage->kind, a, n_cus, s);
  if (!rc) HIP_TRY(hipEventRecord(ev1, s));
  HIP_TRY(hipStreamSynchronize(s));
  float ms = 0.f;
  if (!rc) HIP_TRY(hipEventElapsedTime(&ms, ev0, ev1));
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  if (rc) return rc;
  uint32_t abort_flag = 0;
  if ((rc = d2h(&abort_flag, &ctl->abort, 4))) return rc;
  if (abort_flag) {
    uint32_t diag[3] = {0, 0, 0};
    (void)d2h(diag, &ctl->diag_arrived, sizeof diag);
    return fail(CAMELOT_ETIMEDOUT,
                "grid barrier timed out (stage kind %d, %d rows, %d CUs at %d, %d workgroups): group %u had "
                "%u arrivals, top counter %u",
                stage->kind, rows, n_cus, cu_offset, kWgPerCu * n_cus, diag[2], diag[0] & 0xffff, diag[0] >> 16);
  }
  // HIP events on the stream the kernel ran on: the whole launch, divided by reps
  if (ns_per_rep) *ns_per_rep = (double)ms * 1e6 / reps;
  if (device_ns_per_rep) {
    uint64_t tr[2] = {0, 0};
    if ((rc = d2h(tr, &ctl->ticks_bench, sizeof tr))) return rc;
    *device_ns_per_rep = tr[1] ? (double)tr[0] * 1e9 / (double)dev.wclk_hz / (double)tr[1] : 0.0;
  }
  return CAMELOT_OK;
}

// ==================================================================== pipelines
struct Ring {
  uint8_t* buf = nullptr;          // device
  uint64_t* state = nullptr;       // device (agent scope) or pinned host (system scope)
  bool state_host = false;
  int depth = 0;
  int64_t stride = 0;
};

// Header at the start of an exported ring's allocation (written by the exporting
// process, read and checked by the importing one): the geometry both sides must
// agree on. The state words follow it, then the slots.
struct IpcRingHeader {
  uint64_t magic;
  int32_t version, depth;
  int64_t stride, side_off, row_bytes;
  int32_t side_bytes, max_batch, stamp_next, pad;
};
constexpr uint64_t kIpcMagic = 0x474e495254454d43ull;      // "CMETRING"
constexpr int32_t kIpcVersion = 1;
constexpr int64_t kIpcHeaderBytes = 256;
constexpr int64_t kIpcMaxBytes = 2LL << 30;                 // an opened allocation stays under 2 GiB
// Exported allocations are whole multiples of 2 MiB: a smaller one may be carved out
// of a larger block the runtime holds, which another process cannot open.
constexpr int64_t kIpcGranule = 2LL << 20;
static_assert(sizeof(IpcRingHeader) <= kIpcHeaderBytes, "ring header");
static_assert(sizeof(hipIpcMemHandle_t) == CAMELOT_IPC_HANDLE_BYTES, "IPC handle size");

struct camelot_pipeline {
  camelot_pipeline_config cfg;
  DevInfo dev;
  int S = 0;
  int64_t in_b[kMaxStages] = {0}, out_b[kMaxStages] = {0};
  int64_t side_off[kMaxStages] = {0};  // offset of boundary i's side plane in a slot
  int k_out = 1;
  // workers: the instances of every stage, stage by stage (worker w runs stage
  // w_stage[w]; stage i's instances are workers first_w[i] .. first_w[i] + n_inst[i] - 1)
  int NW = 0;
  int n_inst[kMaxStages] = {0}, first_w[kMaxStages] = {0}, w_stage[kMaxWorkers] = {0};
  int w_off[kMaxWorkers] = {0};    // first CU mask bit of each worker's share
  StageRes res[kMaxWorkers];
  hipStream_t streams[kMaxWorkers] = {nullptr};
  WorkerArgs args[kMaxWorkers];
  WorkerCtl* ctl[kMaxWorkers] = {nullptr};
  // device-global rings (DEVICE handoff: one per boundary; HOST: producer + consumer side)
  Ring out_ring[kMaxStages];       // written by stage i
  Ring in_ring[kMaxStages];        // read by stage i (== out_ring[i-1] in DEVICE mode)
  // host-staged relay
  std::vector<std::thread> relays;
  hipStream_t relay_stream[kMaxStages] = {nullptr};
  uint8_t* staging[kMaxStages] = {nullptr};
  // control blocks (pinned)
  HostCtl* hctl = nullptr;
  DevPub* pub = nullptr;
  // ingest (host mode: pinned ring; replay: device table)
  IngestRec* ingest = nullptr;
  uint8_t* ingest_payload = nullptr;
  int64_t ingest_slot_bytes = 0;
  IngestRec* replay_tab = nullptr;
  uint64_t head = 0;               // requests published (host mode)
  uint64_t last_id = 0;
  bool any_id = false;
  uint64_t submitted_rows = 0, submitted_req = 0;
  // egress
  uint8_t* egress = nullptr;
  int rec_bytes = 0;
  uint64_t egress_tail = 0;
  // clock mapping
  int64_t calib_host_ns = 0;
  int64_t calib_dev_ticks = 0;
  int64_t epoch_ticks = 0;
  bool launched = false;
  bool stopped = false;
  int64_t footprint = 0;
  std::atomic<bool> relay_stop{false};
  // paced host submission (camelot_pipeline_submit_replay)
  std::thread submitter;
  std::atomic<bool> submit_stop{false};
  std::atomic<int32_t> submit_rc{0};
  std::atomic<int64_t> submit_count{0};
  // cross-process rings: the last stage's exported output ring (out_ipc) and the
  // first stage's input ring opened from another process (CAMELOT_INGEST_IPC)
  uint8_t* ipc_out_base = nullptr;         // this process's allocation, exported
  uint8_t* ipc_in_base = nullptr;          // another process's allocation, opened
  uint8_t ipc_handle[CAMELOT_IPC_HANDLE_BYTES] = {0};
  int64_t ipc_setup_ns = 0;
  IpcRingHeader ipc_in_hdr = {};           // geometry of the opened ring
  int stamp_base = 0;                      // index of stage 0 in the timestamps
};


static void* pinned(size_t bytes) {
  void* p = nullptr;
  if (hipHostMalloc(&p, bytes, hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess) return nullptr;
  std::memset(p, 0, bytes);
  return p;
}

static int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

__global__ void camelot_read_clock(uint64_t* out) {
  if (threadIdx.x == 0) *out = (uint64_t)wall_clock64();
}

static int32_t calibrate_clock(camelot_pipeline* p) {
  uint64_t* hp = (uint64_t*)pinned(64);
  if (!hp) return fail(CAMELOT_ENOMEM, "pinned allocation failed");
  hipStream_t s;
  HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  int64_t best_span = INT64_MAX;
  for (int i = 0; i < 5; ++i) {
    const int64_t h0 = host_ns();
    hipLaunchKernelGGL(camelot_read_clock, dim3(1), dim3(64), 0, s, hp);
    if (hipStreamSynchronize(s) != hipSuccess) break;
    const int64_t h1 = host_ns();
    if (h1 - h0 < best_span) {
      best_span = h1 - h0;
      p->calib_host_ns = (h0 + h1) / 2;
      p->calib_dev_ticks = (int64_t)*(volatile uint64_t*)hp;
    }
  }
  (void)hipStreamDestroy(s);
  (void)hipHostFree(hp);
  return CAMELOT_OK;
}

static int64_t host_now_ticks(const camelot_pipeline* p) {
  return p->calib_dev_ticks + ns_to_ticks(host_ns() - p->calib_host_ns, p->dev.wclk_hz);
}

static void relay_loop(camelot_pipeline* p, int i) {
  // boundary i: stage i writes out_ring[i] (device payload, pinned states),
  // stage i+1 reads in_ring[i+1].
  Ring& A = p->out_ring[i];
  Ring& B = p->in_ring[i + 1];
  volatile uint64_t* sa = A.state;
  volatile uint64_t* sb = B.state;
  const int D = A.depth;
  hipStream_t s = p->relay_stream[i];
  for (uint64_t seq = 0;; ++seq) {
    const int slot = (int)(seq % D);
    while (__atomic_load_n(&sa[slot], __ATOMIC_ACQUIRE) != 2 * seq + 1) {
      if (p->relay_stop.load()) return;
      std::this_thread::yield();
    }
    const uint64_t rows = __atomic_load_n(&sa[D + slot], __ATOMIC_ACQUIRE);
    // the slot's header and rows, then its side plane (each row's side bytes)
    const int64_t bytes = kSlotHeaderBytes + (int64_t)rows * p->out_b[i];
    const int64_t soff = p->side_off[i], sbytes = (int64_t)rows * p->cfg.side_bytes;
    if (hipMemcpyAsync(p->staging[i], A.buf + slot * A.stride, bytes, hipMemcpyDeviceToHost, s) != hipSuccess ||
        (sbytes > 0 && hipMemcpyAsync(p->staging[i] + soff, A.buf + slot * A.stride + soff, sbytes,
                                      hipMemcpyDeviceToHost, s) != hipSuccess) ||
        hipStreamSynchronize(s) != hipSuccess)
      return;
    __atomic_store_n(&sa[slot], 2 * seq + 2, __ATOMIC_RELEASE);
    const uint64_t want = seq < (uint64_t)D ? 0 : 2 * (seq - D) + 2;
    while (__atomic_load_n(&sb[slot], __ATOMIC_ACQUIRE) != want) {
      if (p->relay_stop.load()) return;
      std::this_thread::yield();
    }
    if (hipMemcpyAsync(B.buf + slot * B.stride, p->staging[i], bytes, hipMemcpyHostToDevice, s) != hipSuccess ||
        (sbytes > 0 && hipMemcpyAsync(B.buf + slot * B.stride + soff, p->staging[i] + soff, sbytes,
                                      hipMemcpyHostToDevice, s) != hipSuccess) ||
        hipStreamSynchronize(s) != hipSuccess)
      return;
    __atomic_store_n(&sb[slot], 2 * seq + 1, __ATOMIC_RELEASE);
  }
}

static void free_pipeline(camelot_pipeline* p) {
  p->relay_stop.store(true);
  for (auto& t : p->relays) if (t.joinable()) t.join();
  for (int w = 0; w < p->NW; ++w) {
    if (p->streams[w]) (void)hipStreamDestroy(p->streams[w]);
    dfree(p->ctl[w]);
  }
  for (int i = 0; i < p->S; ++i) {
    if (p->relay_stream[i]) (void)hipStreamDestroy(p->relay_stream[i]);
    if (p->staging[i]) (void)hipHostFree(p->staging[i]);
    Ring* rs[2] = {&p->out_ring[i], &p->in_ring[i]};
    for (Ring* r : rs) {
      dfree(r->buf);
      if (r->state) { if (r->state_host) (void)hipHostFree(r->state); else dfree(r->state); }
      r->buf = nullptr;
      r->state = nullptr;
    }
    // DEVICE mode shares one ring object between out_ring[i] and in_ring[i+1]
    if (i + 1 < p->S && p->cfg.handoff == CAMELOT_HANDOFF_DEVICE) {
      p->in_ring[i + 1].buf = nullptr;
      p->in_ring[i + 1].state = nullptr;
    }
  }
  if (p->ipc_out_base) (void)hipFree(p->ipc_out_base);
  if (p->ipc_in_base) (void)hipIpcCloseMemHandle(p->ipc_in_base);
  if (p->hctl) (void)hipHostFree(p->hctl);
  if (p->pub) (void)hipHostFree(p->pub);
  if (p->ingest) (void)hipHostFree(p->ingest);
  if (p->ingest_payload) (void)hipHostFree(p->ingest_payload);
  if (p->egress) (void)hipHostFree(p->egress);
  dfree(p->replay_tab);
  (void)hipStreamSynchronize(mem_stream());
  delete p;
}

static int32_t validate_config(const camelot_pipeline_config* c, const DevInfo& dev, camelot_pipeline* p) {
  if (c->n_stages < 1 || c->n_stages > kMaxStages) return fail(CAMELOT_EINVAL, "n_stages must be in 1..%d", kMaxStages);
  int32_t rc;
  int off = c->cu_offset;
  for (int i = 0; i < c->n_stages; ++i) {
    if ((rc = check_stage(&c->stages[i], &p->in_b[i], &p->out_b[i]))) return rc;
    // an exporting pipeline ends in a ring another process reads, not in results
    const bool result_here = i == c->n_stages - 1 && !c->out_ipc;
    if (is_result_stage(c->stages[i].kind) != result_here)
      return fail(CAMELOT_EINVAL,
                  c->out_ipc ? "stage %d: an exporting pipeline (out_ipc) has no result stage (GEMM_ARGMAX, TOPK)"
                             : "stage %d: result stages (GEMM_ARGMAX, TOPK) must be last and the last stage must be one",
                  i);
    if (i > 0 && p->out_b[i - 1] != p->in_b[i])
      return fail(CAMELOT_EINVAL, "stage %d consumes %lld-byte rows but stage %d produces %lld", i,
                  (long long)p->in_b[i], i - 1, (long long)p->out_b[i - 1]);
    const int n = c->n_inst[i] == 0 ? 1 : c->n_inst[i];
    if (n < 1 || n > CAMELOT_MAX_INSTANCES)
      return fail(CAMELOT_EINVAL, "stage %d: instances must be in 1..%d", i, CAMELOT_MAX_INSTANCES);
    if (n > 1 && (i == 0 || i == c->n_stages - 1))
      return fail(CAMELOT_EINVAL, "stage %d: only stages between the first and the last can have several instances", i);
    if (c->ring_depth < 2 * n) return fail(CAMELOT_EINVAL, "ring_depth must be >= 2 x the instances of a stage");
    for (int j = 0; j < n; ++j) {
      if ((rc = check_share(c->cu[i], off, dev.n_cus))) return rc;
      off += c->cu[i];
    }
    p->n_inst[i] = n;
    p->first_w[i] = p->NW;
    for (int j = 0; j < n; ++j) p->w_stage[p->NW++] = i;
  }
  if (p->NW > kMaxWorkers) return fail(CAMELOT_EINVAL, "more than %d stage instances", kMaxWorkers);
  if (c->max_batch < 1 || c->max_batch > kMaxBatch) return fail(CAMELOT_EINVAL, "max_batch must be in 1..%d", kMaxBatch);
  if (c->batch_target < 1) return fail(CAMELOT_EINVAL, "batch_target must be >= 1");
  if (c->batch_timeout_ns < 0) return fail(CAMELOT_EINVAL, "batch_timeout_ns must be >= 0");
  if (c->ring_depth < 2 || c->ring_depth > 1024) return fail(CAMELOT_EINVAL, "ring_depth must be in 2..1024");
  if (c->handoff != CAMELOT_HANDOFF_DEVICE && c->handoff != CAMELOT_HANDOFF_HOST)
    return fail(CAMELOT_EINVAL, "unknown handoff mode");
  if (c->ingest != CAMELOT_INGEST_HOST && c->ingest != CAMELOT_INGEST_REPLAY && c->ingest != CAMELOT_INGEST_IPC)
    return fail(CAMELOT_EINVAL, "unknown ingest mode");
  if (c->out_ipc != 0 && c->out_ipc != 1) return fail(CAMELOT_EINVAL, "out_ipc must be 0 or 1");
  if (c->max_rows_per_request < 1 || c->max_rows_per_request > c->max_batch)
    return fail(CAMELOT_EINVAL, "max_rows_per_request must be in 1..max_batch");
  if (c->ingest == CAMELOT_INGEST_HOST && (c->ingest_capacity < 1 || c->ingest_capacity > (1 << 22)))
    return fail(CAMELOT_EINVAL, "ingest_capacity must be in 1..2^22");
  if (c->egress_capacity < c->max_batch || c->egress_capacity > (1 << 24))
    return fail(CAMELOT_EINVAL, "egress_capacity must be in max_batch..2^24");
  if (c->idle_timeout_ns <= 0) return fail(CAMELOT_EINVAL, "idle_timeout_ns must be > 0");
  if (c->side_bytes < 0 || c->side_bytes > 4096 || c->side_bytes % 16 != 0)
    return fail(CAMELOT_EINVAL, "side_bytes must be a multiple of 16 in 0..4096");
  for (int i = 0; i < c->n_stages; ++i)
    if (c->stages[i].kind == CAMELOT_STAGE_GATHER_SCORE && c->side_bytes < 4 * c->stages[i].dims[2])
      return fail(CAMELOT_EINVAL, "stage %d reads %d ids from the side bytes", i, c->stages[i].dims[2]);
  return CAMELOT_OK;
}

extern "C" int32_t camelot_pipeline_create(const camelot_pipeline_config* cfg, camelot_pipeline** out) {
  clear_error();
  if (!cfg || !out) return fail(CAMELOT_EINVAL, "cfg/out is NULL");
  *out = nullptr;
  auto* p = new camelot_pipeline();
  std::memset(&p->cfg, 0, sizeof p->cfg);
  p->cfg = *cfg;
  int32_t rc = dev_info(&p->dev);
  if (!rc) rc = validate_config(cfg, p->dev, p);
  if (rc) { delete p; return rc; }
  const int S = p->S = cfg->n_stages;
  const int D = cfg->ring_depth;
  const bool host_handoff = cfg->handoff == CAMELOT_HANDOFF_HOST;
  p->k_out = result_k(&cfg->stages[S - 1]);
  p->rec_bytes = (int)round_up(sizeof(EgressRec) + 8LL * p->k_out, 16);

  // ---- footprint (HBM held by the library) and admission
  int64_t fp = 0;
  int64_t stride[kMaxStages] = {0};
  const int64_t side = cfg->side_bytes;
  int64_t side_off[kMaxStages] = {0};
  for (int i = 0; i + 1 < S; ++i) {
    side_off[i] = p->side_off[i] = kSlotHeaderBytes + round_up((int64_t)cfg->max_batch * p->out_b[i], 256);
    stride[i] = side_off[i] + round_up((int64_t)cfg->max_batch * side, 256);
    fp += (host_handoff ? 2 : 1) * (D * stride[i] + (host_handoff ? 0 : round_up(8LL * D, 256)));
  }
  for (int w = 0; w < p->NW; ++w) {
    int st = 0;
    fp += stage_scratch_bytes(&cfg->stages[p->w_stage[w]], &st) + round_up(sizeof(WorkerCtl), 256);
  }
  // the last stage's exported ring (out_ipc): [header | state words | slots]
  int64_t ipc_side_off = 0, ipc_stride = 0, ipc_bytes = 0;
  if (cfg->out_ipc) {
    ipc_side_off = kSlotHeaderBytes + round_up((int64_t)cfg->max_batch * p->out_b[S - 1], 256);
    ipc_stride = ipc_side_off + round_up((int64_t)cfg->max_batch * side, 256);
    ipc_bytes = kIpcHeaderBytes + round_up(8LL * D, 256) + D * ipc_stride;
    if (round_up(ipc_bytes, kIpcGranule) >= kIpcMaxBytes) {
      delete p;
      return fail(CAMELOT_EINVAL, "the exported ring takes %lld bytes; it must stay under 2 GiB (fewer slots)",
                  (long long)ipc_bytes);
    }
    fp += round_up(ipc_bytes, kIpcGranule);
  }
  p->footprint = fp;
  if (cfg->hbm_budget_bytes > 0 && fp > cfg->hbm_budget_bytes) {
    delete p;
    return fail(CAMELOT_ENOMEM, "pipeline needs %lld bytes of HBM, budget %lld", (long long)fp,
                (long long)cfg->hbm_budget_bytes);
  }

#define P_TRY(expr)                                                                 \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess) {                                                         \
      rc = fail(CAMELOT_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));           \
      free_pipeline(p);                                                             \
      return rc;                                                                    \
    }                                                                               \
  } while (0)
#define P_CHECK(cond, msg)                         \
  do {                                             \
    if (!(cond)) {                                 \
      rc = fail(CAMELOT_ENOMEM, "%s", msg);        \
      free_pipeline(p);                            \
      return rc;                                   \
    }                                              \
  } while (0)

  // ---- control blocks
  p->hctl = (HostCtl*)pinned(sizeof(HostCtl));
  p->pub = (DevPub*)pinned(sizeof(DevPub));
  P_CHECK(p->hctl && p->pub, "pinned allocation failed");
  p->egress = (uint8_t*)pinned((size_t)cfg->egress_capacity * p->rec_bytes);
  P_CHECK(p->egress, "pinned egress allocation failed");
  if (cfg->ingest == CAMELOT_INGEST_HOST) {
    p->ingest = (IngestRec*)pinned((size_t)cfg->ingest_capacity * sizeof(IngestRec));
    p->ingest_slot_bytes = round_up((int64_t)cfg->max_rows_per_request * (p->in_b[0] + cfg->side_bytes), 64);
    p->ingest_payload = (uint8_t*)pinned((size_t)cfg->ingest_capacity * p->ingest_slot_bytes);
    P_CHECK(p->ingest && p->ingest_payload, "pinned ingest allocation failed");
  }

  // ---- rings
  for (int i = 0; i + 1 < S; ++i) {
    Ring& o = p->out_ring[i];
    o.depth = D;
    o.stride = stride[i];
    rc = dmalloc(&o.buf, D * stride[i]);
    if (rc) { free_pipeline(p); return rc; }
    if (host_handoff) {
      o.state_host = true;
      o.state = (uint64_t*)pinned(16LL * D);
      P_CHECK(o.state, "pinned ring state allocation failed");
      Ring& in = p->in_ring[i + 1];
      in.depth = D;
      in.stride = stride[i];
      rc = dmalloc(&in.buf, D * stride[i]);
      if (rc) { free_pipeline(p); return rc; }
      in.state_host = true;
      in.state = (uint64_t*)pinned(16LL * D);
      P_CHECK(in.state, "pinned ring state allocation failed");
      p->staging[i] = nullptr;
      P_TRY(hipHostMalloc((void**)&p->staging[i], stride[i], hipHostMallocDefault));
      P_TRY(hipStreamCreateWithFlags(&p->relay_stream[i], hipStreamNonBlocking));
    } else {
      rc = dmalloc(&o.state, round_up(8LL * D, 256));
      if (!rc) rc = dzero(o.state, round_up(8LL * D, 256));
      if (rc) { free_pipeline(p); return rc; }
      p->in_ring[i + 1] = o;
    }
  }

  // ---- cross-process rings: open the input ring first (it fixes where this
  // pipeline's stages sit in the timestamps), then export the output ring
  if (cfg->ingest == CAMELOT_INGEST_IPC) {
    const int64_t t0 = host_ns();
    hipIpcMemHandle_t h;
    std::memcpy(&h, cfg->ipc_handle, sizeof h);
    P_TRY(hipIpcOpenMemHandle((void**)&p->ipc_in_base, h, hipIpcMemLazyEnablePeerAccess));
    IpcRingHeader& hd = p->ipc_in_hdr;
    rc = d2h(&hd, p->ipc_in_base, sizeof hd);
    if (rc) { free_pipeline(p); return rc; }
    const char* bad = hd.magic != kIpcMagic || hd.version != kIpcVersion ? "is not a ring exported by this library"
                      : hd.row_bytes != p->in_b[0] ? "carries rows of another size than stage 0 consumes"
                      : hd.side_bytes != cfg->side_bytes ? "carries another number of side bytes"
                      : hd.max_batch > cfg->max_batch ? "carries batches larger than max_batch"
                      : hd.stamp_next + S > kMaxStages ? "leaves too few stage timestamps for this pipeline"
                                                       : nullptr;
    if (bad) {
      rc = fail(CAMELOT_EINVAL, "the opened ring %s", bad);
      free_pipeline(p);
      return rc;
    }
    p->stamp_base = hd.stamp_next;
    p->ipc_setup_ns += host_ns() - t0;
  }
  if (cfg->out_ipc) {
    const int64_t t0 = host_ns();
    P_TRY(hipMalloc((void**)&p->ipc_out_base, round_up(ipc_bytes, kIpcGranule)));
    P_TRY(hipMemset(p->ipc_out_base, 0, ipc_bytes));
    IpcRingHeader hd = {};
    hd.magic = kIpcMagic;
    hd.version = kIpcVersion;
    hd.depth = D;
    hd.stride = ipc_stride;
    hd.side_off = ipc_side_off;
    hd.row_bytes = p->out_b[S - 1];
    hd.side_bytes = cfg->side_bytes;
    hd.max_batch = cfg->max_batch;
    hd.stamp_next = p->stamp_base + S;
    rc = h2d(p->ipc_out_base, &hd, sizeof hd);
    if (rc) { free_pipeline(p); return rc; }
    hipIpcMemHandle_t h;
    P_TRY(hipIpcGetMemHandle(&h, p->ipc_out_base));
    std::memcpy(p->ipc_handle, &h, sizeof h);
    p->ipc_setup_ns += host_ns() - t0;
  }

  release_cached_streams();
  // ---- stage instance (worker) resources, control, streams
  int off = cfg->cu_offset;
  for (int w = 0; w < p->NW; ++w) {
    const int i = p->w_stage[w];
    const int inst = w - p->first_w[i];
    WorkerArgs& a = p->args[w];
    std::memset(&a, 0, sizeof a);
    rc = fill_params(&cfg->stages[i], &p->res[w], &a.sp);
    if (rc) { free_pipeline(p); return rc; }
    rc = dmalloc(&p->ctl[w], sizeof(WorkerCtl));
    if (!rc) rc = dzero(p->ctl[w], sizeof(WorkerCtl));
    // instance j starts at batch j and takes every n_inst-th batch
    const uint64_t first_seq = (uint64_t)inst;
    if (!rc) rc = h2d(&p->ctl[w]->next_seq, &first_seq, sizeof first_seq);
    if (rc) { free_pipeline(p); return rc; }
    rc = make_masked_stream(off, cfg->cu[i], &p->streams[w]);
    if (rc) { free_pipeline(p); return rc; }
    p->w_off[w] = off;
    off += cfg->cu[i];
    a.stage_index = p->stamp_base + i;
    a.n_stages = S;
    a.worker_index = w;
    a.n_inst = p->n_inst[i];
    a.ctl_wg = 1;             // a worker's last workgroup forms, broadcasts and publishes batches
    a.max_batch = cfg->max_batch;
    a.side_bytes = cfg->side_bytes;
    a.in_row_stride = (int32_t)(p->in_b[i] + cfg->side_bytes);
    a.in_side_off = i > 0 ? side_off[i - 1] : 0;
    a.out_side_off = i + 1 < S ? side_off[i] : 0;
    a.batch_target = std::min(cfg->batch_target, cfg->max_batch);
    a.batch_timeout_ticks = ns_to_ticks(cfg->batch_timeout_ns, p->dev.wclk_hz);
    a.idle_ticks = ns_to_ticks(cfg->idle_timeout_ns, p->dev.wclk_hz);
    a.spin_ticks = 2 * p->dev.wclk_hz;
    if (i == 0 && cfg->ingest == CAMELOT_INGEST_IPC) {
      const IpcRingHeader& hd = p->ipc_in_hdr;
      a.in_kind = kInRing;
      a.in_depth = hd.depth;
      a.in_state = (uint64_t*)(p->ipc_in_base + kIpcHeaderBytes);
      a.in_ring = p->ipc_in_base + kIpcHeaderBytes + round_up(8LL * hd.depth, 256);
      a.in_state_sys = 0;
      a.in_stride = hd.stride;
      a.in_side_off = hd.side_off;
    } else if (i == 0) {
      a.in_kind = cfg->ingest == CAMELOT_INGEST_HOST ? kInHost : kInReplay;
      if (cfg->ingest == CAMELOT_INGEST_HOST) {
        a.ingest = p->ingest;
        a.n_ingest = cfg->ingest_capacity;
        a.ingest_payload = p->ingest_payload;
      }
    } else {
      const Ring& r = p->in_ring[i];
      a.in_kind = kInRing;
      a.in_depth = r.depth;
      a.in_ring = r.buf;
      a.in_state = r.state;
      a.in_state_sys = r.state_host ? 1 : 0;
      a.in_stride = r.stride;
    }
    if (i + 1 < S) {
      const Ring& r = p->out_ring[i];
      a.out_kind = kOutRing;
      a.out_depth = r.depth;
      a.out_ring = r.buf;
      a.out_state = r.state;
      a.out_state_sys = r.state_host ? 1 : 0;
      a.out_stride = r.stride;
    } else if (cfg->out_ipc) {
      a.out_kind = kOutRing;
      a.out_depth = D;
      a.out_state = (uint64_t*)(p->ipc_out_base + kIpcHeaderBytes);
      a.out_ring = p->ipc_out_base + kIpcHeaderBytes + round_up(8LL * D, 256);
      a.out_state_sys = 0;
      a.out_stride = ipc_stride;
      a.out_side_off = ipc_side_off;
    } else {
      a.out_kind = kOutEgress;
      a.egress = p->egress;
      a.egress_cap = cfg->egress_capacity;
      a.rec_bytes = p->rec_bytes;
    }
    a.ctl = p->ctl[w];
    a.hctl = p->hctl;
    a.pub = p->pub;
  }
  rc = calibrate_clock(p);
  if (rc) { free_pipeline(p); return rc; }
  // a pipeline fed by another process keeps the device clock's zero as its epoch, so
  // its results' timestamps (arrivals stamped upstream included) are absolute
  p->epoch_ticks = cfg->ingest == CAMELOT_INGEST_IPC ? 0 : host_now_ticks(p);

  if (host_handoff)
    for (int i = 0; i + 1 < S; ++i) p->relays.emplace_back(relay_loop, p, i);

  if (cfg->ingest == CAMELOT_INGEST_HOST || cfg->ingest == CAMELOT_INGEST_IPC) {
    for (int w = p->NW - 1; w >= 0; --w) {
      const int i = p->w_stage[w];
      rc = launch_worker(cfg->stages[i].kind, p->args[w], cfg->cu[i], p->streams[w]);
      if (rc) { free_pipeline(p); return rc; }
    }
    p->launched = true;
  }
  *out = p;
  return CAMELOT_OK;
#undef P_TRY
#undef P_CHECK
}

extern "C" int64_t camelot_pipeline_footprint(const camelot_pipeline* p) { return p ? p->footprint : -1; }

extern "C" int32_t camelot_pipeline_epoch_ns(const camelot_pipeline* p, int64_t* epoch_ns) {
  clear_error();
  if (!p || !epoch_ns) return fail(CAMELOT_EINVAL, "bad epoch arguments");
  int64_t ticks = p->epoch_ticks;
  if (p->cfg.ingest == CAMELOT_INGEST_REPLAY) {
    ticks = (int64_t)__atomic_load_n(&p->pub->t0, __ATOMIC_ACQUIRE);
    if (!p->launched || ticks == 0) return fail(CAMELOT_EAGAIN, "the replay has not started");
  }
  *epoch_ns = (int64_t)ticks_to_ns(ticks, p->dev.wclk_hz);
  return CAMELOT_OK;
}

extern "C" int32_t camelot_pipeline_ipc_info(const camelot_pipeline* p, uint8_t* handle, int64_t* setup_ns) {
  clear_error();
  if (!p || !handle || !setup_ns) return fail(CAMELOT_EINVAL, "bad ipc_info arguments");
  std::memcpy(handle, p->ipc_handle, CAMELOT_IPC_HANDLE_BYTES);
  *setup_ns = p->ipc_setup_ns;
  if (!p->cfg.out_ipc && p->cfg.ingest != CAMELOT_INGEST_IPC)
    return fail(CAMELOT_EINVAL, "the pipeline neither exports nor imports a ring");
  return CAMELOT_OK;
}

static int32_t worker_error(camelot_pipeline* p) {
  for (int w = 0; w < p->NW; ++w) {
    const int32_t st = __atomic_load_n(&p->pub->status[w], __ATOMIC_ACQUIRE);
    if (st == kStatusTimeout || st == kStatusAborted) {
      // a grid barrier that timed out recorded which counter was short
      uint32_t diag[3] = {0, 0, 0};
      (void)d2h(diag, &p->ctl[w]->diag_arrived, sizeof diag);
      const int i = p->w_stage[w];
      return fail(CAMELOT_EDEVICE,
                  "stage %d worker %d (%d CUs at %d) failed (status %d); barrier diagnostics: %u workgroups, "
                  "group %u had %u arrivals, top counter %u",
                  i, w - p->first_w[i], p->cfg.cu[i], p->w_off[w], st, diag[1], diag[2], diag[0] & 0xffff,
                  diag[0] >> 16);
    }
    if (st == kStatusIdleExit)
      return fail(CAMELOT_ESTOPPED, "stage %d worker exited after the idle timeout", p->w_stage[w]);
  }
  return CAMELOT_OK;
}

static int32_t submit_at(camelot_pipeline* p, uint64_t query_id, const void* payload, int32_t rows,
                         int64_t arrival_host_ns);

extern "C" int32_t camelot_pipeline_submit(camelot_pipeline* p, uint64_t query_id, const void* payload,
                                           int32_t rows) {
  clear_error();
  return submit_at(p, query_id, payload, rows, -1);
}

// Workers that left after the idle timeout start again, from the state they saved at
// exit (batch sequence, ingest cursor, egress head, counters), when new work is
// submitted. Their go words still hold the value of the stop broadcast, which is the
// one the next batch would use, so they are cleared first, on the worker's own
// stream, ahead of the launch.
static int32_t relaunch_idle(camelot_pipeline* p) {
  if (!p->launched || p->stopped) return CAMELOT_OK;
  for (int w = 0; w < p->NW; ++w) {
    if (__atomic_load_n(&p->pub->status[w], __ATOMIC_ACQUIRE) != kStatusIdleExit) continue;
    // the control workgroup publishes the status last; the compute workgroups leave
    // on its stop broadcast
    HIP_TRY(hipStreamSynchronize(p->streams[w]));
    HIP_TRY(hipMemsetAsync(&p->ctl[w]->go, 0, sizeof(p->ctl[w]->go), p->streams[w]));
    __atomic_store_n(&p->pub->started[w], 0, __ATOMIC_RELEASE);
    __atomic_store_n(&p->pub->status[w], (int32_t)kStatusOk, __ATOMIC_RELEASE);
    const int i = p->w_stage[w];
    if (int32_t rc = launch_worker(p->cfg.stages[i].kind, p->args[w], p->cfg.cu[i], p->streams[w])) return rc;
  }
  return CAMELOT_OK;
}

// arrival_host_ns < 0: the query arrives now
static int32_t submit_at(camelot_pipeline* p, uint64_t query_id, const void* payload, int32_t rows,
                         int64_t arrival_host_ns) {
  if (!p) return fail(CAMELOT_EINVAL, "pipeline is NULL");
  if (p->stopped) return fail(CAMELOT_ESTOPPED, "pipeline is stopped");
  if (p->cfg.ingest != CAMELOT_INGEST_HOST) return fail(CAMELOT_EINVAL, "pipeline uses replay ingest");
  if (rows < 1 || rows > p->cfg.max_rows_per_request)
    return fail(CAMELOT_EINVAL, "rows must be in 1..%d", p->cfg.max_rows_per_request);
  if (!payload) return fail(CAMELOT_EINVAL, "payload is NULL");
  if (p->any_id && query_id <= p->last_id) return fail(CAMELOT_EINVAL, "query ids must increase");
  int32_t rc = relaunch_idle(p);
  if (rc) return rc;
  rc = worker_error(p);
  if (rc) return rc;
  const uint64_t tail = __atomic_load_n(&p->pub->ingest_tail, __ATOMIC_ACQUIRE);
  if (p->head - tail >= (uint64_t)p->cfg.ingest_capacity) return fail(CAMELOT_EAGAIN, "ingest queue full");
  const uint64_t slot = p->head % (uint64_t)p->cfg.ingest_capacity;
  std::memcpy(p->ingest_payload + slot * p->ingest_slot_bytes, payload,
              (size_t)rows * (p->in_b[0] + p->cfg.side_bytes));
  IngestRec rec;
  rec.id = query_id;
  rec.t_arr = (uint64_t)(arrival_host_ns < 0
                             ? host_now_ticks(p)
                             : p->calib_dev_ticks + ns_to_ticks(arrival_host_ns - p->calib_host_ns, p->dev.wclk_hz));
  rec.payload_off = slot * (uint64_t)p->ingest_slot_bytes;
  rec.rows = (uint32_t)rows;
  rec.valid = (uint32_t)(p->head / (uint64_t)p->cfg.ingest_capacity + 1);
  std::memcpy(&p->ingest[slot], &rec, sizeof rec);
  ++p->head;
  __atomic_store_n(&p->hctl->ingest_head, p->head, __ATOMIC_RELEASE);
  p->last_id = query_id;
  p->any_id = true;
  p->submitted_rows += rows;
  p->submitted_req += 1;
  return CAMELOT_OK;
}

// The paced submitter: request r goes through the submit path once arrival_ns[r]
// has passed since the call (busy-waiting on the host clock), retried while the
// ingest queue is full, stamped with its scheduled arrival time.
static void submit_loop(camelot_pipeline* p, std::vector<uint64_t> ids, std::vector<int32_t> rows,
                        std::vector<int64_t> arr, std::vector<int64_t> prow, const uint8_t* payload,
                        int64_t row_bytes, int64_t t0) {
  for (size_t r = 0; r < ids.size(); ++r) {
    const int64_t due = t0 + arr[r];
    while (host_ns() < due)
      if (p->submit_stop.load(std::memory_order_relaxed)) return;
    for (;;) {
      // the query's arrival is its scheduled time: a submitter that falls behind
      // shows up in the latencies, not hidden by a later stamp
      const int32_t rc = submit_at(p, ids[r], payload + prow[r] * row_bytes, rows[r], due);
      if (rc == CAMELOT_OK) break;
      if (rc != CAMELOT_EAGAIN || p->submit_stop.load(std::memory_order_relaxed)) {
        p->submit_rc.store(rc);
        return;
      }
      std::this_thread::yield();
    }
    p->submit_count.store((int64_t)r + 1, std::memory_order_relaxed);
  }
}

static void stop_submitter(camelot_pipeline* p) {
  if (p->submitter.joinable()) {
    p->submit_stop.store(true);
    p->submitter.join();
  }
}

extern "C" int32_t camelot_pipeline_submit_replay(camelot_pipeline* p, int32_t n_req, const uint64_t* ids,
                                                  const int32_t* rows, const int64_t* arrival_ns,
                                                  const int64_t* payload_row, const void* payload,
                                                  int64_t payload_rows) {
  clear_error();
  if (!p) return fail(CAMELOT_EINVAL, "pipeline is NULL");
  if (p->cfg.ingest != CAMELOT_INGEST_HOST) return fail(CAMELOT_EINVAL, "pipeline uses replay ingest");
  if (p->submitter.joinable()) return fail(CAMELOT_EINVAL, "a paced submission already ran on this pipeline");
  if (n_req < 0 || (n_req > 0 && (!ids || !rows || !arrival_ns || !payload_row || !payload)))
    return fail(CAMELOT_EINVAL, "replay arrays are NULL");
  for (int r = 0; r < n_req; ++r) {
    if (rows[r] < 1 || rows[r] > p->cfg.max_rows_per_request)
      return fail(CAMELOT_EINVAL, "request %d: rows must be in 1..%d", r, p->cfg.max_rows_per_request);
    if ((r > 0 && ids[r] <= ids[r - 1]) || (p->any_id && ids[r] <= p->last_id))
      return fail(CAMELOT_EINVAL, "request ids must increase");
    if (arrival_ns[r] < 0 || (r > 0 && arrival_ns[r] < arrival_ns[r - 1]))
      return fail(CAMELOT_EINVAL, "arrival times must be non-decreasing and >= 0");
    if (payload_row[r] < 0 || payload_row[r] + rows[r] > payload_rows)
      return fail(CAMELOT_EINVAL, "request %d: payload rows outside the buffer", r);
  }
  p->submit_rc.store(0);
  p->submit_count.store(0);
  p->submit_stop.store(false);
  p->submitter = std::thread(submit_loop, p, std::vector<uint64_t>(ids, ids + n_req),
                             std::vector<int32_t>(rows, rows + n_req), std::vector<int64_t>(arrival_ns, arrival_ns + n_req),
                             std::vector<int64_t>(payload_row, payload_row + n_req), (const uint8_t*)payload,
                             p->in_b[0] + p->cfg.side_bytes, host_ns());
  return CAMELOT_OK;
}

extern "C" int32_t camelot_pipeline_submit_status(camelot_pipeline* p, int64_t* submitted) {
  clear_error();
  if (!p || !submitted) return fail(CAMELOT_EINVAL, "bad status arguments");
  *submitted = p->submit_count.load();
  const int32_t rc = p->submit_rc.load();
  return rc ? fail(rc, "paced submission stopped with error %d after %lld requests", rc, (long long)*submitted)
            : CAMELOT_OK;
}

extern "C" int32_t camelot_pipeline_replay(camelot_pipeline* p, int32_t n_req, const uint64_t* ids,
                                           const int32_t* rows, const int64_t* arrival_ns,
                                           const int64_t* payload_row, const void* payload,
                                           int64_t payload_rows) {
  clear_error();
  if (!p) return fail(CAMELOT_EINVAL, "pipeline is NULL");
  if (p->cfg.ingest != CAMELOT_INGEST_REPLAY) return fail(CAMELOT_EINVAL, "pipeline uses host ingest");
  if (p->launched) return fail(CAMELOT_EINVAL, "replay already started");
  if (n_req < 0 || (n_req > 0 && (!ids || !rows || !arrival_ns || !payload_row || !payload)))
    return fail(CAMELOT_EINVAL, "replay arrays are NULL");
  std::vector<IngestRec> tab((size_t)std::max(n_req, 1));
  for (int r = 0; r < n_req; ++r) {
    if (rows[r] < 1 || rows[r] > p->cfg.max_rows_per_request)
      return fail(CAMELOT_EINVAL, "request %d: rows must be in 1..%d", r, p->cfg.max_rows_per_request);
    if (r > 0 && ids[r] <= ids[r - 1]) return fail(CAMELOT_EINVAL, "request ids must increase");
    if (arrival_ns[r] < 0 || (r > 0 && arrival_ns[r] < arrival_ns[r - 1]))
      return fail(CAMELOT_EINVAL, "arrival times must be non-decreasing and >= 0");
    if (payload_row[r] < 0 || payload_row[r] + rows[r] > payload_rows)
      return fail(CAMELOT_EINVAL, "request %d: payload rows out of range", r);
    tab[r].id = ids[r];
    tab[r].t_arr = (uint64_t)ns_to_ticks(arrival_ns[r], p->dev.wclk_hz);
    tab[r].payload_off = (uint64_t)payload_row[r] * (uint64_t)(p->in_b[0] + p->cfg.side_bytes);
    tab[r].rows = (uint32_t)rows[r];
    tab[r].valid = 1;
    p->submitted_rows += rows[r];
  }
  p->submitted_req = (uint64_t)n_req;
  int32_t rc0 = dmalloc(&p->replay_tab, tab.size() * sizeof(IngestRec));
  if (!rc0) rc0 = h2d(p->replay_tab, tab.data(), tab.size() * sizeof(IngestRec));
  if (rc0) return rc0;
  // arrival times are relative; stage 0 adds the epoch it takes at start
  p->args[0].ingest = p->replay_tab;
  p->args[0].n_ingest = n_req;
  p->args[0].ingest_payload = (const uint8_t*)payload;
  for (int w = p->NW - 1; w >= 0; --w) {
    const int i = p->w_stage[w];
    int32_t rc = launch_worker(p->cfg.stages[i].kind, p->args[w], p->cfg.cu[i], p->streams[w]);
    if (rc) return rc;
  }
  p->launched = true;
  return CAMELOT_OK;
}

// Waits (bounded) until the egress record at position pos carries its sequence word:
// the device writes it after the record's other fields are acknowledged.
static int32_t await_record(camelot_pipeline* p, uint64_t pos, const uint8_t* rec) {
  const uint64_t* seq = (const uint64_t*)(rec + offsetof(EgressRec, seq));
  if (__atomic_load_n(seq, __ATOMIC_ACQUIRE) == pos + 1) return CAMELOT_OK;
  const int64_t t_end = host_ns() + 1000000000LL;
  while (__atomic_load_n(seq, __ATOMIC_ACQUIRE) != pos + 1) {
    if (host_ns() > t_end) {
      const EgressRec* h = (const EgressRec*)rec;
      return fail(CAMELOT_EDEVICE,
                  "egress record %llu published without its contents (sequence word %llu, id %llu, row %u, "
                  "egress head %llu, tail %llu)",
                  (unsigned long long)pos, (unsigned long long)__atomic_load_n(seq, __ATOMIC_ACQUIRE),
                  (unsigned long long)h->id, h->row,
                  (unsigned long long)__atomic_load_n(&p->pub->egress_head, __ATOMIC_ACQUIRE),
                  (unsigned long long)p->egress_tail);
    }
    std::this_thread::yield();
  }
  return CAMELOT_OK;
}

extern "C" int32_t camelot_pipeline_drain(camelot_pipeline* p, camelot_result* out, int32_t max,
                                          int32_t* n_out, int64_t timeout_ns) {
  clear_error();
  if (!p || !out || !n_out || max < 0) return fail(CAMELOT_EINVAL, "bad drain arguments");
  if (p->cfg.out_ipc) return fail(CAMELOT_EINVAL, "the pipeline exports its batches; results come out of the importing one");
  *n_out = 0;
  const int64_t t_end = host_ns() + std::max<int64_t>(timeout_ns, 0);
  uint64_t head;
  for (;;) {
    head = __atomic_load_n(&p->pub->egress_head, __ATOMIC_ACQUIRE);
    if (head > p->egress_tail || max == 0) break;
    int32_t rc = worker_error(p);
    if (rc && rc != CAMELOT_ESTOPPED) return rc;
    if (host_ns() >= t_end) {
      if (rc == CAMELOT_ESTOPPED) return rc;
      return fail(CAMELOT_ETIMEDOUT, "no result within the timeout");
    }
    std::this_thread::yield();
  }
  const uint64_t n = std::min<uint64_t>(head - p->egress_tail, (uint64_t)max);
  // the stages of upstream processes come first in the timestamps
  const int S = p->stamp_base + p->S;
  const int64_t epoch = p->cfg.ingest == CAMELOT_INGEST_REPLAY
                            ? (int64_t)__atomic_load_n(&p->pub->t0, __ATOMIC_ACQUIRE)
                            : p->epoch_ticks;
  const int64_t hz = p->dev.wclk_hz;
  for (uint64_t j = 0; j < n; ++j) {
    const uint64_t slot = (p->egress_tail + j) % (uint64_t)p->cfg.egress_capacity;
    const uint8_t* rec = p->egress + slot * p->rec_bytes;
    if (int32_t rc = await_record(p, p->egress_tail + j, rec)) return rc;
    EgressRec h;
    std::memcpy(&h, rec, sizeof h);
    camelot_result& r = out[j];
    std::memset(&r, 0, sizeof r);
    r.query_id = h.id;
    r.row = (int32_t)h.row;
    r.n_out = (int32_t)h.n_out;
    std::memcpy(r.idx, rec + sizeof(EgressRec), 4LL * p->k_out);
    std::memcpy(r.val, rec + sizeof(EgressRec) + 4LL * p->k_out, 4LL * p->k_out);
    r.t_ns[0] = ticks_to_ns((int64_t)h.t_arr - epoch, hz);
    for (int s = 0; s < S; ++s) {
      r.t_ns[1 + 2 * s] = ticks_to_ns((int64_t)h.t_stage[2 * s] - epoch, hz);
      r.t_ns[2 + 2 * s] = ticks_to_ns((int64_t)h.t_stage[2 * s + 1] - epoch, hz);
    }
    r.t_ns[2 * S] = ticks_to_ns((int64_t)h.t_done - epoch, hz);   // last stage ends when its row is done
    r.t_ns[2 * S + 1] = ticks_to_ns((int64_t)h.t_done - epoch, hz);
  }
  p->egress_tail += n;
  __atomic_store_n(&p->hctl->egress_tail, p->egress_tail, __ATOMIC_RELEASE);
  *n_out = (int32_t)n;
  return CAMELOT_OK;
}

extern "C" int32_t camelot_pipeline_drain_latency(camelot_pipeline* p, uint64_t* ids, int64_t* lat_ns,
                                                  int32_t max, int32_t* n_out, int64_t timeout_ns) {
  clear_error();
  if (!p || !ids || !lat_ns || !n_out || max < 0) return fail(CAMELOT_EINVAL, "bad drain arguments");
  if (p->cfg.out_ipc) return fail(CAMELOT_EINVAL, "the pipeline exports its batches; results come out of the importing one");
  *n_out = 0;
  const int64_t t_end = host_ns() + std::max<int64_t>(timeout_ns, 0);
  uint64_t head;
  for (;;) {
    head = __atomic_load_n(&p->pub->egress_head, __ATOMIC_ACQUIRE);
    if (head > p->egress_tail || max == 0) break;
    int32_t rc = worker_error(p);
    if (rc && rc != CAMELOT_ESTOPPED) return rc;
    if (host_ns() >= t_end) {
      if (rc == CAMELOT_ESTOPPED) return rc;
      return fail(CAMELOT_ETIMEDOUT, "no result within the timeout");
    }
    std::this_thread::yield();
  }
  const uint64_t n = std::min<uint64_t>(head - p->egress_tail, (uint64_t)max);
  const int64_t hz = p->dev.wclk_hz;
  for (uint64_t j = 0; j < n; ++j) {
    const uint64_t slot = (p->egress_tail + j) % (uint64_t)p->cfg.egress_capacity;
    const EgressRec* h = (const EgressRec*)(p->egress + slot * p->rec_bytes);
    if (int32_t rc = await_record(p, p->egress_tail + j, (const uint8_t*)h)) return rc;
    ids[j] = h->id;
    lat_ns[j] = (int64_t)ticks_to_ns((int64_t)h->t_done - (int64_t)h->t_arr, hz);
  }
  p->egress_tail += n;
  __atomic_store_n(&p->hctl->egress_tail, p->egress_tail, __ATOMIC_RELEASE);
  *n_out = (int32_t)n;
  return CAMELOT_OK;
}

extern "C" int32_t camelot_pipeline_stats_get(camelot_pipeline* p, camelot_pipeline_stats* out) {
  clear_error();
  if (!p || !out) return fail(CAMELOT_EINVAL, "bad arguments");
  std::memset(out, 0, sizeof *out);
  out->submitted_requests = p->submitted_req;
  out->submitted_rows = p->submitted_rows;
  out->delivered_rows = __atomic_load_n(&p->pub->egress_head, __ATOMIC_ACQUIRE);
  // per stage: sums over its instances (the id checksums are sums and xors, so the
  // instances' partial values combine exactly)
  for (int w = 0; w < p->NW; ++w) {
    const int i = p->w_stage[w];
    out->batches[i] += __atomic_load_n(&p->pub->batches[w], __ATOMIC_ACQUIRE);
    out->id_sum[i] += __atomic_load_n(&p->pub->id_sum[w], __ATOMIC_ACQUIRE);
    out->id_xor[i] ^= __atomic_load_n(&p->pub->id_xor[w], __ATOMIC_ACQUIRE);
    const int32_t st = __atomic_load_n(&p->pub->status[w], __ATOMIC_ACQUIRE);
    if (out->worker_status[i] == 0) out->worker_status[i] = st;
    out->rows[i] += __atomic_load_n(&p->pub->rows[w], __ATOMIC_ACQUIRE);
    out->busy_ns[i] += ticks_to_ns((int64_t)__atomic_load_n(&p->pub->busy_ticks[w], __ATOMIC_ACQUIRE), p->dev.wclk_hz);
    out->wait_ns[i] += ticks_to_ns((int64_t)__atomic_load_n(&p->pub->wait_ticks[w], __ATOMIC_ACQUIRE), p->dev.wclk_hz);
  }
  return CAMELOT_OK;
}

extern "C" int32_t camelot_pipeline_destroy(camelot_pipeline* p, uint64_t* undelivered) {
  clear_error();
  if (!p) return fail(CAMELOT_EINVAL, "pipeline is NULL");
  stop_submitter(p);
  p->stopped = true;
  __atomic_store_n(&p->hctl->stop, 1ull, __ATOMIC_RELEASE);
  int32_t rc = CAMELOT_OK;
  if (p->launched) {
    // workers poll the stop flag between batches; in-batch waits are bounded
    const int64_t deadline = host_ns() + 30LL * 1000000000LL;
    for (int i = 0; i < p->NW; ++i) {
      for (;;) {
        hipError_t q = hipStreamQuery(p->streams[i]);
        if (q == hipSuccess) break;
        if (q != hipErrorNotReady) { rc = fail(CAMELOT_EDEVICE, "stage %d stream: %s", i, hipGetErrorString(q)); break; }
        if (host_ns() > deadline) {
          // the worker still runs: its memory cannot be released safely
          p->relay_stop.store(true);
          for (auto& t : p->relays) if (t.joinable()) t.join();
          return fail(CAMELOT_ETIMEDOUT, "stage %d worker did not stop; pipeline memory leaked", i);
        }
        std::this_thread::sleep_for(std::chrono::microseconds(50));
      }
    }
  }
  const uint64_t delivered = __atomic_load_n(&p->pub->egress_head, __ATOMIC_ACQUIRE);
  if (undelivered) *undelivered = p->submitted_rows > delivered ? p->submitted_rows - delivered : 0;
  free_pipeline(p);
  return rc;
}

// ==================================================================== handoff benchmark

static void expected_checksum(int64_t slot_bytes, int64_t n_slots, uint64_t* sum, uint64_t* xr) {
  // sum / xor over s < n_slots, w < W of (s * 0x9E3779B1 mod 2^32) xor w, bit by bit
  const uint64_t W = (uint64_t)(slot_bytes / 4);
  uint64_t ones[32];
  for (int b = 0; b < 32; ++b) {
    const uint64_t period = 1ull << (b + 1), half = 1ull << b;
    ones[b] = (W / period) * half + (W % period > half ? W % period - half : 0);
  }
  uint64_t s_acc = 0, x_acc = 0;
  for (int64_t s = 0; s < n_slots; ++s) {
    const uint32_t c = (uint32_t)((uint64_t)s * 0x9E3779B1ull);
    for (int b = 0; b < 32; ++b) {
      const uint64_t cnt = ((c >> b) & 1u) ? W - ones[b] : ones[b];
      s_acc += cnt << b;
      if (cnt & 1) x_acc ^= 1ull << b;
    }
  }
  *sum = s_acc;
  *xr = x_acc;
}

extern "C" int32_t camelot_handoff_expected(int64_t slot_bytes, int64_t n_slots_total, uint64_t* sum,
                                            uint64_t* xr) {
  clear_error();
  if (slot_bytes < 16 || slot_bytes % 16 != 0 || n_slots_total < 0 || !sum || !xr)
    return fail(CAMELOT_EINVAL, "slot_bytes must be a positive multiple of 16");
  expected_checksum(slot_bytes, n_slots_total, sum, xr);
  return CAMELOT_OK;
}

extern "C" int32_t camelot_handoff_bench(int32_t mode, int64_t slot_bytes, int32_t depth, int64_t n_slots,
                                         int32_t cu_producer, int32_t cu_consumer, double* out) {
  clear_error();
  if (!out) return fail(CAMELOT_EINVAL, "out is NULL");
  if (slot_bytes < 16 || slot_bytes % 16 != 0 || slot_bytes > (1LL << 30) || depth < 1 || n_slots < 1)
    return fail(CAMELOT_EINVAL, "slot_bytes must be a multiple of 16 in 16..2^30; depth, n_slots >= 1");
  DevInfo dev;
  int32_t rc = dev_info(&dev);
  if (rc) return rc;
  std::memset(out, 0, 5 * sizeof(double));
  if (mode == CAMELOT_HANDOFF_HOST) {
    uint8_t *src = nullptr, *dst = nullptr, *host = nullptr;
    hipStream_t s;
    if ((rc = dmalloc(&src, slot_bytes * depth)) || (rc = dmalloc(&dst, slot_bytes * depth))) return rc;
    HIP_TRY(hipHostMalloc((void**)&host, slot_bytes, hipHostMallocDefault));
    HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    HIP_TRY(hipMemsetAsync(src, 1, slot_bytes * depth, s));
    HIP_TRY(hipStreamSynchronize(s));
    const int64_t t0 = host_ns();
    for (int64_t i = 0; i < n_slots; ++i) {
      const int64_t d = i % depth;
      HIP_TRY(hipMemcpyAsync(host, src + d * slot_bytes, slot_bytes, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipMemcpyAsync(dst + d * slot_bytes, host, slot_bytes, hipMemcpyHostToDevice, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    const int64_t t1 = host_ns();
    (void)hipStreamDestroy(s);
    dfree(src);
    dfree(dst);
    (void)hipStreamSynchronize(mem_stream());
    (void)hipHostFree(host);
    out[0] = (t1 - t0) * 1e-9;
    out[1] = 2.0 * (double)slot_bytes * (double)n_slots;
    out[4] = out[1] / out[0] / 1e9;
    return CAMELOT_OK;
  }
  if (mode != CAMELOT_HANDOFF_DEVICE) return fail(CAMELOT_EINVAL, "unknown handoff mode");
  if ((rc = check_share(cu_producer, 0, dev.n_cus))) return rc;
  if ((rc = check_share(cu_consumer, cu_producer, dev.n_cus))) return rc;
  const int nwg = kWgPerCu * std::min(cu_producer, cu_consumer);
  int64_t chunk = (slot_bytes + nwg - 1) / nwg;
  chunk = round_up(chunk, 16);
  hipStream_t sp, sc;
  if ((rc = cached_stream(0, cu_producer, &sp))) return rc;
  if ((rc = cached_stream(cu_producer, cu_consumer, &sc))) return rc;
  HandoffArgs a;
  std::memset(&a, 0, sizeof a);
  if ((rc = dmalloc(&a.ring, slot_bytes * depth)) || (rc = dmalloc(&a.full, 4LL * depth * nwg)) ||
      (rc = dmalloc(&a.freed, 4LL * depth * nwg)) || (rc = dmalloc(&a.result, 64)) ||
      (rc = dzero(a.full, 4LL * depth * nwg)) || (rc = dzero(a.freed, 4LL * depth * nwg)))
    return rc;
  uint64_t init[8] = {0, 0, ~0ull, 0, 0, 0, 0, 0};
  if ((rc = h2d(a.result, init, 64))) return rc;
  a.slot_bytes = slot_bytes;
  a.depth = depth;
  a.n_slots = n_slots;
  a.chunk_bytes = chunk;
  a.spin_ticks = 2 * dev.wclk_hz;
  void* args[] = {(void*)&a};
  HIP_TRY(hipLaunchKernel((const void*)camelot_handoff_consumer, dim3(nwg), dim3(kThreads), args, 0, sc));
  HIP_TRY(hipLaunchKernel((const void*)camelot_handoff_producer, dim3(nwg), dim3(kThreads), args, 0, sp));
  HIP_TRY(hipStreamSynchronize(sp));
  HIP_TRY(hipStreamSynchronize(sc));
  uint64_t r[8];
  rc = d2h(r, a.result, 64);
  dfree(a.ring);
  dfree(a.full);
  dfree(a.freed);
  dfree(a.result);
  (void)hipStreamSynchronize(mem_stream());
  if (rc) return rc;
  if (r[4]) return fail(CAMELOT_ETIMEDOUT, "handoff channel wait timed out");
  out[0] = (double)(r[3] - r[2]) / (double)dev.wclk_hz;
  out[1] = 2.0 * (double)slot_bytes * (double)n_slots;
  out[2] = (double)r[0];
  out[3] = (double)r[1];
  out[4] = out[1] / out[0] / 1e9;
  // exact checksums are returned bit-for-bit through the double slots' bytes
  std::memcpy(&out[2], &r[0], 8);
  std::memcpy(&out[3], &r[1], 8);
  return CAMELOT_OK;
}

// ==================================================================== cross-process handoff benchmark
// The handoff kernels above with their ring, doorbells and results in one device
// allocation that a second process opens: the producer runs in one process, the
// consumer in the other, on the same GPU.
struct IpcRegionHeader {
  uint64_t magic;
  int32_t version, depth, nwg, pad;
  int64_t slot_bytes, chunk_bytes;
};
constexpr uint64_t kIpcRegionMagic = 0x4e4f494745524d43ull;   // "CMREGION"

struct camelot_ipc_region {
  uint8_t* base = nullptr;
  bool owner = false;
  IpcRegionHeader h = {};
  int64_t setup_ns = 0;
};

// [header 256 | results 64 | full: depth x nwg words | freed: same | ring: depth slots]
static int64_t region_full_off() { return 256 + 64; }
static int64_t region_freed_off(const IpcRegionHeader& h) { return region_full_off() + round_up(4LL * h.depth * h.nwg, 256); }
static int64_t region_ring_off(const IpcRegionHeader& h) { return region_freed_off(h) + round_up(4LL * h.depth * h.nwg, 256); }

extern "C" int32_t camelot_ipc_region_create(int64_t slot_bytes, int32_t depth, int32_t channels, uint8_t* handle,
                                             camelot_ipc_region** out) {
  clear_error();
  if (!handle || !out) return fail(CAMELOT_EINVAL, "handle/out is NULL");
  *out = nullptr;
  if (slot_bytes < 16 || slot_bytes % 16 != 0 || depth < 1 || channels < 1 || channels > 256)
    return fail(CAMELOT_EINVAL, "slot_bytes must be a positive multiple of 16, depth >= 1, channels in 1..256");
  IpcRegionHeader h = {};
  h.magic = kIpcRegionMagic;
  h.version = kIpcVersion;
  h.depth = depth;
  h.slot_bytes = slot_bytes;
  // every channel (workgroup pair) owns a chunk of each slot, at least 16 bytes
  const int64_t want = std::min<int64_t>(channels, slot_bytes / 16);
  h.chunk_bytes = round_up((slot_bytes + want - 1) / want, 16);
  h.nwg = (int32_t)((slot_bytes + h.chunk_bytes - 1) / h.chunk_bytes);
  const int64_t bytes = region_ring_off(h) + (int64_t)depth * slot_bytes;
  if (round_up(bytes, kIpcGranule) >= kIpcMaxBytes) return fail(CAMELOT_EINVAL, "the region takes %lld bytes; it must stay under 2 GiB",
                                         (long long)bytes);
  DevInfo dev;                                    // the runtime is up before the clock starts
  if (int32_t rc = dev_info(&dev)) return rc;
  const int64_t t0 = host_ns();
  auto* r = new camelot_ipc_region();
  r->owner = true;
  r->h = h;
  hipError_t e = hipMalloc((void**)&r->base, round_up(bytes, kIpcGranule));
  if (e == hipSuccess) e = hipMemset(r->base, 0, bytes);
  uint64_t init[8] = {0, 0, ~0ull, 0, 0, 0, 0, 0};      // sum, xor, first start (min), last end (max), error
  if (e == hipSuccess) e = hipMemcpy(r->base, &h, sizeof h, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(r->base + 256, init, sizeof init, hipMemcpyHostToDevice);
  hipIpcMemHandle_t ih;
  if (e == hipSuccess) e = hipIpcGetMemHandle(&ih, r->base);
  if (e != hipSuccess) {
    if (r->base) (void)hipFree(r->base);
    delete r;
    return fail(CAMELOT_EDEVICE, "IPC region: %s", hipGetErrorString(e));
  }
  std::memcpy(handle, &ih, sizeof ih);
  r->setup_ns = host_ns() - t0;
  *out = r;
  return CAMELOT_OK;
}

extern "C" int32_t camelot_ipc_region_open(const uint8_t* handle, camelot_ipc_region** out) {
  clear_error();
  if (!handle || !out) return fail(CAMELOT_EINVAL, "handle/out is NULL");
  *out = nullptr;
  DevInfo dev;                                    // the runtime is up before the clock starts
  if (int32_t rc = dev_info(&dev)) return rc;
  const int64_t t0 = host_ns();
  hipIpcMemHandle_t ih;
  std::memcpy(&ih, handle, sizeof ih);
  auto* r = new camelot_ipc_region();
  hipError_t e = hipIpcOpenMemHandle((void**)&r->base, ih, hipIpcMemLazyEnablePeerAccess);
  if (e == hipSuccess) e = hipMemcpy(&r->h, r->base, sizeof r->h, hipMemcpyDeviceToHost);
  if (e != hipSuccess) {
    if (r->base) (void)hipIpcCloseMemHandle(r->base);
    delete r;
    return fail(CAMELOT_EDEVICE, "IPC region open: %s", hipGetErrorString(e));
  }
  if (r->h.magic != kIpcRegionMagic || r->h.version != kIpcVersion) {
    (void)hipIpcCloseMemHandle(r->base);
    delete r;
    return fail(CAMELOT_EINVAL, "the opened allocation is not a handoff region of this library");
  }
  r->setup_ns = host_ns() - t0;
  *out = r;
  return CAMELOT_OK;
}

extern "C" int32_t camelot_ipc_region_info(const camelot_ipc_region* r, int64_t* setup_ns, int32_t* channels) {
  clear_error();
  if (!r || !setup_ns || !channels) return fail(CAMELOT_EINVAL, "bad region_info arguments");
  *setup_ns = r->setup_ns;
  *channels = r->h.nwg;
  return CAMELOT_OK;
}

extern "C" int32_t camelot_ipc_handoff_run(camelot_ipc_region* r, int32_t role, int64_t n_slots, int32_t cu_offset,
                                           int32_t timeout_ms, double* out) {
  clear_error();
  if (!r || !out) return fail(CAMELOT_EINVAL, "region/out is NULL");
  if (role != CAMELOT_IPC_PRODUCER && role != CAMELOT_IPC_CONSUMER) return fail(CAMELOT_EINVAL, "unknown role");
  if (n_slots < 1 || timeout_ms < 1 || timeout_ms > 600000)
    return fail(CAMELOT_EINVAL, "n_slots >= 1; timeout_ms in 1..600000");
  DevInfo dev;
  int32_t rc = dev_info(&dev);
  if (rc) return rc;
  const int n_cus = (int)round_up(r->h.nwg, 8);
  if ((rc = check_share(n_cus, cu_offset, dev.n_cus))) return rc;
  std::memset(out, 0, 5 * sizeof(double));
  hipStream_t s;
  if ((rc = cached_stream(cu_offset, n_cus, &s))) return rc;
  HandoffArgs a;
  std::memset(&a, 0, sizeof a);
  a.result = (uint64_t*)(r->base + 256);
  a.full = (uint32_t*)(r->base + region_full_off());
  a.freed = (uint32_t*)(r->base + region_freed_off(r->h));
  a.ring = r->base + region_ring_off(r->h);
  a.slot_bytes = r->h.slot_bytes;
  a.depth = r->h.depth;
  a.n_slots = n_slots;
  a.chunk_bytes = r->h.chunk_bytes;
  a.spin_ticks = (int64_t)timeout_ms * (dev.wclk_hz / 1000);
  void* args[] = {(void*)&a};
  const void* fn = role == CAMELOT_IPC_PRODUCER ? (const void*)camelot_handoff_producer
                                                : (const void*)camelot_handoff_consumer;
  HIP_TRY(hipLaunchKernel(fn, dim3(r->h.nwg), dim3(kThreads), args, 0, s));
  HIP_TRY(hipStreamSynchronize(s));
  uint64_t res[8];
  if ((rc = d2h(res, a.result, 64))) return rc;
  if (res[4]) return fail(CAMELOT_ETIMEDOUT, "handoff channel wait timed out (the other side did not keep up)");
  out[0] = res[3] > res[2] ? (double)(res[3] - res[2]) / (double)dev.wclk_hz : 0.0;
  out[1] = 2.0 * (double)r->h.slot_bytes * (double)n_slots;
  std::memcpy(&out[2], &res[0], 8);
  std::memcpy(&out[3], &res[1], 8);
  out[4] = out[0] > 0 ? out[1] / out[0] / 1e9 : 0.0;
  return CAMELOT_OK;
}

extern "C" int32_t camelot_ipc_region_destroy(camelot_ipc_region* r) {
  clear_error();
  if (!r) return fail(CAMELOT_EINVAL, "region is NULL");
  hipError_t e = r->owner ? hipFree(r->base) : hipIpcCloseMemHandle(r->base);
  delete r;
  if (e != hipSuccess) return fail(CAMELOT_EDEVICE, "IPC region release: %s", hipGetErrorString(e));
  return CAMELOT_OK;
}

// ==================================================================== predictor
extern "C" __global__ void camelot_pred_forward(const float*, const float*, int, float*);
extern "C" __global__ void camelot_pred_grad_partial(const float*, const float*, const float*, const int32_t*, int,
                                                     float*);
extern "C" __global__ void camelot_pred_grad_reduce(const float*, int, int, float*, float*);
extern "C" __global__ void camelot_pred_adam(float*, const float*, float*, float*, float, float, float);

namespace {
struct PredWork {
  float* partial = nullptr;
  int cap = 0;   // workgroups
  float* loss = nullptr;
};
PredWork g_pw;

int32_t pred_work(int nwg) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (nwg > g_pw.cap) {
    dfree(g_pw.partial);
    g_pw.partial = nullptr;
    int32_t rc = dmalloc(&g_pw.partial, 4LL * nwg * (CAMELOT_PRED_NPARAMS + 1));
    if (rc) return rc;
    g_pw.cap = nwg;
  }
  if (!g_pw.loss) {
    int32_t rc = dmalloc(&g_pw.loss, 4 * 1024);
    if (rc) return rc;
  }
  return CAMELOT_OK;
}

int32_t grad_launch(const float* params, const float* x, const float* y, const int32_t* idx, int m, float* grad,
                    float* loss_dev, hipStream_t s) {
  const int nwg = (m + 63) / 64;
  int32_t rc = pred_work(nwg);
  if (rc) return rc;
  hipLaunchKernelGGL(camelot_pred_grad_partial, dim3(nwg), dim3(kThreads), 0, s, params, x, y, idx, m, g_pw.partial);
  hipLaunchKernelGGL(camelot_pred_grad_reduce, dim3((CAMELOT_PRED_NPARAMS + 1 + kThreads - 1) / kThreads),
                     dim3(kThreads), 0, s, (const float*)g_pw.partial, nwg, m, grad, loss_dev);
  HIP_TRY(hipGetLastError());
  return CAMELOT_OK;
}
}  // namespace

extern "C" int32_t camelot_predictor_forward(const float* params, const float* x, int32_t m, float* yhat,
                                             void* stream) {
  clear_error();
  if (!params || !x || !yhat || m < 0) return fail(CAMELOT_EINVAL, "bad predictor arguments");
  if (m == 0) return CAMELOT_OK;
  hipStream_t s = stream ? (hipStream_t)stream : mem_stream();
  hipLaunchKernelGGL(camelot_pred_forward, dim3((m + kThreads - 1) / kThreads), dim3(kThreads), 0, s, params, x, m,
                     yhat);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  return CAMELOT_OK;
}

extern "C" int32_t camelot_predictor_grad(const float* params, const float* x, const float* y, int32_t m,
                                          float* grad, float* loss_out, void* stream) {
  clear_error();
  if (!params || !x || !y || !grad || m < 1) return fail(CAMELOT_EINVAL, "bad predictor arguments");
  hipStream_t s = stream ? (hipStream_t)stream : mem_stream();
  int32_t rc = pred_work((m + 63) / 64);
  if (rc) return rc;
  if ((rc = grad_launch(params, x, y, nullptr, m, grad, g_pw.loss, s))) return rc;
  HIP_TRY(hipStreamSynchronize(s));
  if (loss_out && (rc = d2h(loss_out, g_pw.loss, 4))) return rc;
  return CAMELOT_OK;
}

extern "C" int32_t camelot_predictor_adam(float* params, const float* grad, float* m1, float* m2, int32_t t,
                                          float lr, void* stream) {
  clear_error();
  if (!params || !grad || !m1 || !m2 || t < 1) return fail(CAMELOT_EINVAL, "bad Adam arguments");
  hipStream_t s = stream ? (hipStream_t)stream : mem_stream();
  const float c1 = (float)(1.0 - std::pow(0.9, (double)t));
  const float c2 = (float)(1.0 - std::pow(0.999, (double)t));
  hipLaunchKernelGGL(camelot_pred_adam, dim3((CAMELOT_PRED_NPARAMS + kThreads - 1) / kThreads), dim3(kThreads), 0, s,
                     params, grad, m1, m2, lr, c1, c2);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  return CAMELOT_OK;
}

extern "C" int32_t camelot_predictor_train(float* params, float* m1, float* m2, int32_t* t, const float* x,
                                           const float* y, int32_t n, int32_t batch, int32_t epochs,
                                           const int32_t* perm, float lr, float* epoch_loss, void* stream) {
  clear_error();
  if (!params || !m1 || !m2 || !t || !x || !y || n < 1 || batch < 1 || epochs < 0 || *t < 0)
    return fail(CAMELOT_EINVAL, "bad training arguments");
  hipStream_t s = stream ? (hipStream_t)stream : mem_stream();
  const int steps_per_epoch = (n + batch - 1) / batch;
  const int total = steps_per_epoch * epochs;
  float* grad = nullptr;
  float* losses = nullptr;
  int32_t rc = dmalloc(&grad, 4 * CAMELOT_PRED_NPARAMS);
  if (!rc) rc = dmalloc(&losses, 4LL * std::max(total, 1));
  if (rc) return rc;
  int step = 0;
  for (int e = 0; e < epochs && !rc; ++e) {
    for (int b = 0; b < steps_per_epoch && !rc; ++b) {
      const int r0 = b * batch;
      const int m = std::min(batch, n - r0);
      const int32_t* idx = perm ? perm + (int64_t)e * n + r0 : nullptr;
      const float* xb = perm ? x : x + (int64_t)r0 * CAMELOT_PRED_NIN;
      const float* yb = perm ? y : y + r0;
      rc = grad_launch(params, xb, yb, idx, m, grad, losses + step, s);
      if (rc) break;
      const int tt = ++(*t);
      const float c1 = (float)(1.0 - std::pow(0.9, (double)tt));
      const float c2 = (float)(1.0 - std::pow(0.999, (double)tt));
      hipLaunchKernelGGL(camelot_pred_adam, dim3((CAMELOT_PRED_NPARAMS + kThreads - 1) / kThreads), dim3(kThreads),
                         0, s, params, (const float*)grad, m1, m2, lr, c1, c2);
      ++step;
    }
  }
  if (!rc && hipStreamSynchronize(s) != hipSuccess) rc = fail(CAMELOT_EDEVICE, "training kernels failed");
  if (!rc && epoch_loss && total > 0) {
    std::vector<float> l((size_t)total);
    if ((rc = d2h(l.data(), losses, 4LL * total)) == CAMELOT_OK) {
      for (int e = 0; e < epochs; ++e) {
        double acc = 0;
        for (int b = 0; b < steps_per_epoch; ++b) acc += l[(size_t)e * steps_per_epoch + b];
        epoch_loss[e] = (float)(acc / steps_per_epoch);
      }
    }
  }
  dfree(grad);
  dfree(losses);
  (void)hipStreamSynchronize(mem_stream());
  return rc;
}
