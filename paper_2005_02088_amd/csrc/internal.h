// Helpers shared by the host-side translation units of libcamelot.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "../../include/camelot.h"
#include "device_common.h"
#include "errors.h"

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return camelot::fail(CAMELOT_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

namespace camelot {

struct DevInfo {
  bool ok = false;
  int n_cus = 0;
  int64_t wclk_hz = 100000000;
  int64_t mem = 0;
  char arch[32] = {0};
};

// Device resources one stage worker needs (scratch, tables). Owned by a pipeline or
// by a one-shot run.
struct StageRes {
  uint16_t* scratch = nullptr;
  int64_t scratch_bytes = 0;
  ~StageRes();
};


int32_t dev_info(DevInfo* out);
hipStream_t mem_stream();
int32_t dmalloc(void** ptr, size_t bytes);
template <typename T>
int32_t dmalloc(T** ptr, size_t bytes) { return dmalloc((void**)ptr, bytes); }
void dfree(void* ptr);
int32_t dzero(void* ptr, size_t bytes);
int32_t d2h(void* dst, const void* src, size_t bytes);
int32_t h2d(void* dst, const void* src, size_t bytes);
int64_t ns_to_ticks(int64_t ns, int64_t hz);
int32_t cached_stream(int offset, int n, hipStream_t* s);
// A new CU-masked stream the caller owns (and destroys).
int32_t new_masked_stream(int offset, int n, hipStream_t* s);
int32_t fill_params(const camelot_stage_desc* d, StageRes* res, StageParams* sp);
// The allocation-free part of fill_params: checks the descriptor and fills sp except
// its device buffers; *scratch_bytes = the stage scratch the kernel needs (0: none).
int32_t stage_params(const camelot_stage_desc* d, StageParams* sp, int64_t* scratch_bytes);
// Points sp at its scratch buffer (MLP hidden state, conv partial sums) and, for
// LOGMEL, at the device copy of the log-mel tables.
void stage_params_bind(StageParams* sp, void* scratch, const float* logmel_tab);
// Window, FFT twiddles and HTK mel filterbank of the LOGMEL stage, computed in double
// and stored as float into t[kLogmelTableFloats]; false if they do not fit.
constexpr int kLogmelTableFloats = 2304;
bool logmel_tables(float* t);

int32_t check_share(int n_cus, int offset, int total);
int32_t launch_worker(int kind, const WorkerArgs& a, int n_cus, hipStream_t s);
bool is_result_stage(int kind);
// Side bytes following each input row in a one-shot run (GATHER_SCORE: its ids).
int64_t stage_side_bytes(const camelot_stage_desc* d);

}  // namespace camelot
