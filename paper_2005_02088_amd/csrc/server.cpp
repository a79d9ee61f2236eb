// Serving: a set of co-located pipelines admitted under one HBM budget, with weight
// buffers shared by pointer counted once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "internal.h"

struct camelot_server {
  int64_t budget = 0;
  int64_t used = 0;
  std::mutex mu;
  struct Member {
    camelot_pipeline* p;
    int64_t own;                       // library footprint
    std::vector<const void*> weights;  // distinct weight buffers it holds a reference on
    int lo, hi;                        // CU-mask bits [lo, hi)
  };
  std::vector<Member> members;
  std::map<const void*, std::pair<int64_t, int>> weights;   // pointer -> (bytes, references)
};

namespace {
using namespace camelot;

int64_t weight_bytes(const camelot_stage_desc* d, std::vector<std::pair<const void*, int64_t>>* parts) {
  auto add = [&](const void* p, int64_t b) {
    if (parts) parts->push_back({p, b});
    return b;
  };
  switch (d->kind) {
    case CAMELOT_STAGE_GEMM_RELU:
    case CAMELOT_STAGE_GEMM_ARGMAX:
      return add(d->weights[0], 4LL * d->dims[0] * d->dims[1]);
    case CAMELOT_STAGE_MLP_BF16: {
      int64_t t = 0;
      for (int l = 0; l < d->n_layers; ++l) t += add(d->weights[l], 2LL * d->dims[l] * d->dims[l + 1]);
      return t;
    }
    case CAMELOT_STAGE_GATHER:
    case CAMELOT_STAGE_GATHER_SCORE:
      return add(d->weights[0], 2LL * d->k * d->dims[1]);
    case CAMELOT_STAGE_CONV_POOL:
      return add(d->weights[0], 2LL * d->dims[3] * 9 * d->dims[2]);
    case CAMELOT_STAGE_ARTIFACT_M:            // the device table (P's lives in host memory)
      return add(d->weights[0], 4LL * d->k);
    default:
      return 0;
  }
}
}  // namespace

extern "C" int64_t camelot_stage_weight_bytes(const camelot_stage_desc* stage) {
  clear_error();
  int64_t i = 0, o = 0;
  int32_t rc = camelot_stage_row_bytes_in(stage);
  if (rc < 0) return rc;
  (void)i;
  (void)o;
  return weight_bytes(stage, nullptr);
}

extern "C" int32_t camelot_server_create(int64_t hbm_budget_bytes, camelot_server** out) {
  clear_error();
  if (!out || hbm_budget_bytes <= 0) return fail(CAMELOT_EINVAL, "budget must be > 0");
  auto* s = new camelot_server();
  s->budget = hbm_budget_bytes;
  *out = s;
  return CAMELOT_OK;
}

extern "C" int32_t camelot_server_admit(camelot_server* s, const camelot_pipeline_config* cfg,
                                        camelot_pipeline** out) {
  clear_error();
  if (!s || !cfg || !out) return fail(CAMELOT_EINVAL, "bad admission arguments");
  std::lock_guard<std::mutex> lk(s->mu);
  int lo = cfg->cu_offset, hi = cfg->cu_offset;
  for (int i = 0; i < cfg->n_stages && i < CAMELOT_MAX_STAGES; ++i)
    hi += cfg->cu[i] * (cfg->n_inst[i] > 1 ? cfg->n_inst[i] : 1);
  for (auto& m : s->members)
    if (lo < m.hi && m.lo < hi) return fail(CAMELOT_EINVAL, "CU range [%d, %d) overlaps an admitted pipeline", lo, hi);
  // weights not yet held
  std::vector<std::pair<const void*, int64_t>> parts;
  for (int i = 0; i < cfg->n_stages && i < CAMELOT_MAX_STAGES; ++i) weight_bytes(&cfg->stages[i], &parts);
  std::map<const void*, int64_t> fresh;
  for (auto& pw : parts)
    if (!s->weights.count(pw.first)) fresh[pw.first] = pw.second;
  int64_t new_w = 0;
  for (auto& f : fresh) new_w += f.second;
  // the pipeline's own footprint, checked against what is left before anything is allocated
  camelot_pipeline_config c = *cfg;
  const int64_t left = s->budget - s->used - new_w;
  if (left <= 0)
    return fail(CAMELOT_ENOMEM, "weights need %lld bytes, %lld left", (long long)new_w,
                (long long)(s->budget - s->used));
  c.hbm_budget_bytes = cfg->hbm_budget_bytes > 0 ? std::min(cfg->hbm_budget_bytes, left) : left;
  camelot_pipeline* p = nullptr;
  int32_t rc = camelot_pipeline_create(&c, &p);
  if (rc) return rc;
  camelot_server::Member m;
  m.p = p;
  m.own = camelot_pipeline_footprint(p);
  m.lo = lo;
  m.hi = hi;
  for (auto& pw : parts) {
    if (std::find(m.weights.begin(), m.weights.end(), pw.first) != m.weights.end()) continue;
    m.weights.push_back(pw.first);
    auto it = s->weights.find(pw.first);
    if (it == s->weights.end()) s->weights[pw.first] = {pw.second, 1};
    else it->second.second += 1;
  }
  s->used += m.own + new_w;
  s->members.push_back(m);
  *out = p;
  return CAMELOT_OK;
}

static int32_t release_locked(camelot_server* s, size_t idx, uint64_t* undelivered) {
  camelot_server::Member m = s->members[idx];
  s->members.erase(s->members.begin() + (long)idx);
  int64_t freed = m.own;
  for (const void* w : m.weights) {
    auto it = s->weights.find(w);
    if (it == s->weights.end()) continue;
    if (--it->second.second == 0) {
      freed += it->second.first;
      s->weights.erase(it);
    }
  }
  s->used -= freed;
  return camelot_pipeline_destroy(m.p, undelivered);
}

extern "C" int32_t camelot_server_release(camelot_server* s, camelot_pipeline* p, uint64_t* undelivered) {
  clear_error();
  if (!s || !p) return fail(CAMELOT_EINVAL, "bad release arguments");
  std::lock_guard<std::mutex> lk(s->mu);
  for (size_t i = 0; i < s->members.size(); ++i)
    if (s->members[i].p == p) return release_locked(s, i, undelivered);
  return fail(CAMELOT_EINVAL, "pipeline is not admitted on this server");
}

extern "C" int64_t camelot_server_used_bytes(const camelot_server* s) { return s ? s->used : -1; }

extern "C" int32_t camelot_server_destroy(camelot_server* s) {
  clear_error();
  if (!s) return fail(CAMELOT_EINVAL, "server is NULL");
  int32_t rc = CAMELOT_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    // stop every pipeline first so no live worker waits behind another's teardown
    while (!s->members.empty()) {
      int32_t r = release_locked(s, s->members.size() - 1, nullptr);
      if (r && !rc) rc = r;
    }
  }
  delete s;
  return rc;
}
