// Contention profiles and the learned contention predictor's host side:
// concurrent co-location runs, random co-location profiling, the 16 features,
// their standardisation, and the contention-aware allocator (Eq. 1 with predicted
// latencies).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <numeric>
#include <vector>

#include "internal.h"

extern "C" __global__ void camelot_pred_forward(const float*, const float*, int, float*);

namespace {

using namespace camelot;

struct CtlBuf {
  WorkerCtl* p = nullptr;
  ~CtlBuf() { dfree(p); }
};

bool overlaps(int a0, int an, int b0, int bn) { return a0 < b0 + bn && b0 < a0 + an; }

uint64_t splitmix_next(uint64_t& s) {
  s += 0x9E3779B97F4A7C15ull;
  uint64_t z = s;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
// uniform integer in [0, n)
int uniform(uint64_t& s, int n) { return (int)(splitmix_next(s) % (uint64_t)n); }

// runs of the co-location walk between two fresh draws
constexpr int kWalkRestart = 16;

}  // namespace

namespace {
// The co-location run on caller-provided CU-masked streams (streams[j] masked to
// n_cus[j] CUs at cu_offset[j]).
int32_t corun_on(int32_t n, const camelot_stage_desc* stages, const void* const* in, void* const* out,
                 const int32_t* rows, const int32_t* n_cus, int64_t duration_ns, double* ns_per_batch,
                 const hipStream_t* streams) {
  DevInfo dev;
  int32_t rc = dev_info(&dev);
  if (rc) return rc;
  std::vector<StageRes> res(n);
  std::vector<CtlBuf> ctl(n);
  std::vector<WorkerArgs> args(n);
  for (int j = 0; j < n; ++j) {
    WorkerArgs& a = args[j];
    std::memset(&a, 0, sizeof a);
    if ((rc = fill_params(&stages[j], &res[j], &a.sp))) return rc;
    if ((rc = dmalloc(&ctl[j].p, sizeof(WorkerCtl))) || (rc = dzero(ctl[j].p, sizeof(WorkerCtl)))) return rc;
    a.n_stages = 1;
    a.max_batch = kMaxBatch;
    a.spin_ticks = 2 * dev.wclk_hz;
    a.idle_ticks = 2 * dev.wclk_hz;
    a.in_kind = kInBench;
    a.out_kind = is_result_stage(stages[j].kind) ? kOutBench : kOutRing;
    a.ctl = ctl[j].p;
    a.bench_in = (const uint8_t*)in[j];
    a.bench_out = (uint8_t*)out[j];
    a.bench_rows = rows[j];
    a.side_bytes = stages[j].kind == CAMELOT_STAGE_GATHER_SCORE ? 4 * stages[j].dims[2] : 0;
    a.in_row_stride = a.sp.in_row_bytes + a.side_bytes;
    a.bench_reps = 1 << 30;
    a.bench_ticks = ns_to_ticks(duration_ns, dev.wclk_hz);
  }
  for (int j = 0; j < n && !rc; ++j) rc = launch_worker(stages[j].kind, args[j], n_cus[j], streams[j]);
  for (int j = 0; j < n; ++j) (void)hipStreamSynchronize(streams[j]);
  if (rc) return rc;
  for (int j = 0; j < n; ++j) {
    uint64_t tr[2] = {0, 0};
    uint32_t abort_flag = 0;
    if ((rc = d2h(tr, &ctl[j].p->ticks_bench, sizeof tr)) || (rc = d2h(&abort_flag, &ctl[j].p->abort, 4)))
      return rc;
    if (abort_flag) return fail(CAMELOT_ETIMEDOUT, "co-run stage %d: grid barrier timed out", j);
    ns_per_batch[j] = tr[1] ? (double)tr[0] * 1e9 / (double)dev.wclk_hz / (double)tr[1] : 0.0;
  }
  return CAMELOT_OK;
}

struct OwnStreams {
  std::vector<hipStream_t> s;
  ~OwnStreams() {
    for (hipStream_t x : s)
      if (x) (void)hipStreamDestroy(x);
  }
};
}  // namespace

extern "C" int32_t camelot_stage_corun(int32_t n, const camelot_stage_desc* stages, const void* const* in,
                                       void* const* out, const int32_t* rows, const int32_t* n_cus,
                                       const int32_t* cu_offset, int64_t duration_ns, double* ns_per_batch) {
  clear_error();
  if (n < 1 || n > kMaxStages || !stages || !in || !out || !rows || !n_cus || !cu_offset || !ns_per_batch)
    return fail(CAMELOT_EINVAL, "bad co-run arguments");
  if (duration_ns <= 0 || duration_ns > 10LL * 1000000000LL)
    return fail(CAMELOT_EINVAL, "duration_ns must be in (0, 10 s]");
  DevInfo dev;
  int32_t rc = dev_info(&dev);
  if (rc) return rc;
  for (int j = 0; j < n; ++j) {
    if ((rc = check_share(n_cus[j], cu_offset[j], dev.n_cus))) return rc;
    if (rows[j] < 0 || rows[j] > kMaxBatch) return fail(CAMELOT_EINVAL, "rows must be in 0..%d", kMaxBatch);
    for (int q = 0; q < j; ++q)
      if (overlaps(cu_offset[j], n_cus[j], cu_offset[q], n_cus[q]))
        return fail(CAMELOT_EINVAL, "co-run shares %d and %d overlap", q, j);
  }
  // own streams (a co-run can hold more kernels than the cache keeps streams)
  OwnStreams own;
  own.s.assign(n, nullptr);
  for (int j = 0; j < n; ++j)
    if ((rc = new_masked_stream(cu_offset[j], n_cus[j], &own.s[j]))) return rc;
  return corun_on(n, stages, in, out, rows, n_cus, duration_ns, ns_per_batch, own.s.data());
}

namespace {
// One kernel of the co-location walk: its kind, share and offset (in CU steps),
// batch index, and the stream masked to its share.
struct WalkKernel {
  int kind, sh, off, bi;
  hipStream_t s;
};

// Free gaps (offset, length in steps) of [0, steps) around the kernels.
std::vector<std::pair<int, int>> free_gaps(const std::vector<WalkKernel>& ks, int steps) {
  std::vector<std::pair<int, int>> used;
  for (const auto& k : ks) used.push_back({k.off, k.sh});
  std::sort(used.begin(), used.end());
  std::vector<std::pair<int, int>> gaps;
  int at = 0;
  for (const auto& u : used) {
    if (u.first > at) gaps.push_back({at, u.first - at});
    at = u.first + u.second;
  }
  if (at < steps) gaps.push_back({at, steps - at});
  return gaps;
}
}  // namespace

extern "C" int32_t camelot_profile_coruns(int32_t n_kinds, const camelot_stage_desc* stages, const void* const* in,
                                          void* const* out, int32_t cu_total, int32_t cu_step, int32_t n_batches,
                                          const int32_t* batches, int32_t n_runs, uint64_t seed,
                                          int64_t duration_ns, camelot_corun_record* records) {
  clear_error();
  if (n_kinds < 1 || n_kinds > 3 || !stages || !in || !out || !batches || n_batches < 1 || n_runs < 0 ||
      !records || cu_step < 8 || cu_step % 8 != 0 || cu_total < cu_step * n_kinds)
    return fail(CAMELOT_EINVAL, "bad co-run profiling arguments");
  DevInfo dev;
  int32_t rc = dev_info(&dev);
  if (rc) return rc;
  if ((rc = check_share(cu_total, 0, dev.n_cus))) return rc;
  uint64_t st = seed;
  const int steps = cu_total / cu_step;
  const int mmax = std::min(CAMELOT_MAX_CORUN, steps);
  std::vector<WalkKernel> ks;
  struct Release {
    std::vector<WalkKernel>* ks;
    ~Release() {
      for (auto& k : *ks)
        if (k.s) (void)hipStreamDestroy(k.s);
    }
  } release{&ks};
  auto drop = [&](size_t i) {
    if (ks[i].s) (void)hipStreamDestroy(ks[i].s);
    ks.erase(ks.begin() + (long)i);
  };
  auto batch_for = [&](bool same) {
    return (same && !ks.empty()) ? ks[uniform(st, (int)ks.size())].bi : uniform(st, n_batches);
  };
  for (int r = 0; r < n_runs; ++r) {
    if (r % kWalkRestart == 0) {
      // a fresh draw: m kernels, shares uniform with total <= the GPU, side by side
      while (!ks.empty()) drop(ks.size() - 1);
      const int m = 1 + uniform(st, mmax);
      int sh[CAMELOT_MAX_CORUN];
      for (;;) {
        int tot = 0;
        for (int i = 0; i < m; ++i) { sh[i] = 1 + uniform(st, steps - (m - 1)); tot += sh[i]; }
        if (tot <= steps) break;
      }
      const bool same = uniform(st, 2) == 0;
      const int b0 = uniform(st, n_batches);
      const bool shaped = m >= n_kinds && uniform(st, 2) == 0;
      int off = 0;
      for (int i = 0; i < m; ++i) {
        const int k = (shaped && i < n_kinds) ? i : uniform(st, n_kinds);
        ks.push_back({k, sh[i], off, same ? b0 : uniform(st, n_batches), nullptr});
        off += sh[i];
      }
    } else {
      // one move of the walk: re-draw a kernel's kind and batch (its share kept),
      // re-draw its share inside the gap it sits in, add a kernel in a free gap, or
      // remove one
      const auto gaps = free_gaps(ks, steps);
      const int move = uniform(st, 4);
      if (move == 0 || (move == 2 && (gaps.empty() || (int)ks.size() >= mmax)) || (move == 3 && ks.size() < 2)) {
        WalkKernel& k = ks[uniform(st, (int)ks.size())];
        k.kind = uniform(st, n_kinds);
        k.bi = batch_for(uniform(st, 2) == 0);
      } else if (move == 1) {
        const size_t i = (size_t)uniform(st, (int)ks.size());
        // the span the kernel may take: its own steps plus the free gap right after it
        int room = ks[i].sh;
        for (const auto& g : gaps)
          if (g.first == ks[i].off + ks[i].sh) room += g.second;
        const int sh = 1 + uniform(st, room);
        if (sh != ks[i].sh) {
          if (ks[i].s) (void)hipStreamDestroy(ks[i].s);
          ks[i].s = nullptr;
          ks[i].sh = sh;
        }
      } else if (move == 2) {
        const auto& g = gaps[(size_t)uniform(st, (int)gaps.size())];
        const int bi = batch_for(uniform(st, 2) == 0);
        ks.push_back({uniform(st, n_kinds), 1 + uniform(st, g.second), g.first, bi, nullptr});
      } else {
        drop((size_t)uniform(st, (int)ks.size()));
      }
    }
    const int m = (int)ks.size();
    camelot_corun_record& rec = records[r];
    std::memset(&rec, 0, sizeof rec);
    rec.m = m;
    camelot_stage_desc d[CAMELOT_MAX_CORUN];
    const void* ins[CAMELOT_MAX_CORUN];
    void* outs[CAMELOT_MAX_CORUN];
    int32_t rows[CAMELOT_MAX_CORUN], cus[CAMELOT_MAX_CORUN];
    hipStream_t ss[CAMELOT_MAX_CORUN];
    for (int i = 0; i < m; ++i) {
      WalkKernel& k = ks[(size_t)i];
      if (!k.s && (rc = new_masked_stream(k.off * cu_step, k.sh * cu_step, &k.s))) return rc;
      rec.kinds[i] = k.kind;
      rec.cu[i] = k.sh * cu_step;
      rec.bi[i] = k.bi;
      d[i] = stages[k.kind];
      ins[i] = in[k.kind];
      outs[i] = out[k.kind];
      rows[i] = batches[k.bi];
      cus[i] = rec.cu[i];
      ss[i] = k.s;
    }
    if ((rc = corun_on(m, d, ins, outs, rows, cus, duration_ns, rec.ns, ss))) return rc;
  }
  return CAMELOT_OK;
}

// ------------------------------------------------------------------ features
namespace {
int32_t check_tables(const camelot_solo_tables* t) {
  if (!t || t->n_kinds < 1 || t->n_kinds > 3 || t->cu_step < 1 || t->n_shares < 1 || t->n_batches < 1 ||
      !t->batches || !t->hbm || !t->mfma)
    return fail(CAMELOT_EINVAL, "bad solo tables");
  return CAMELOT_OK;
}

inline float log2b(int b) { return std::log2((float)std::max(b, 1)) / 7.f; }

// one row of 16 features for kernel j of a co-location (no validation)
void feature_row(const camelot_solo_tables* t, int m, const int32_t* kinds, const int32_t* cu,
                 const int32_t* bi, int j, float* f) {
  auto at = [&](const float* tab, int k, int share_cus, int b) {
    const int ks = share_cus / t->cu_step - 1;
    return tab[((int64_t)k * t->n_shares + ks) * t->n_batches + b];
  };
  std::memset(f, 0, CAMELOT_PRED_FEATURES * sizeof(float));
  f[0] = cu[j] / 256.f;
  f[1] = log2b(t->batches[bi[j]]);
  f[2] = at(t->hbm, kinds[j], cu[j], bi[j]);
  f[3] = at(t->mfma, kinds[j], cu[j], bi[j]);
  f[4 + kinds[j]] = 1.f;
  // slot 0 (features 7..10): the other instances of kind[j]; slot 1 (11..14): the
  // kernels of other kinds
  int cnt[2] = {0, 0}, total = 0;
  for (int q = 0; q < m; ++q) {
    total += cu[q];
    if (q == j) continue;
    const int slot = kinds[q] == kinds[j] ? 0 : 1;
    float* g = f + 7 + 4 * slot;
    g[0] += cu[q] / 256.f;
    g[1] += log2b(t->batches[bi[q]]);
    g[2] += at(t->hbm, kinds[q], cu[q], bi[q]);
    g[3] += at(t->mfma, kinds[q], cu[q], bi[q]);
    ++cnt[slot];
  }
  for (int slot = 0; slot < 2; ++slot)
    if (cnt[slot] > 1) f[7 + 4 * slot + 1] /= (float)cnt[slot];
  f[15] = total / 256.f;
}
}  // namespace

extern "C" int32_t camelot_predictor_features(const camelot_solo_tables* t, int32_t m, const int32_t* kinds,
                                              const int32_t* cu, const int32_t* bi, float* feat) {
  clear_error();
  int32_t rc = check_tables(t);
  if (rc) return rc;
  if (m < 1 || m > CAMELOT_MAX_CORUN || !kinds || !cu || !bi || !feat)
    return fail(CAMELOT_EINVAL, "bad feature arguments");
  for (int j = 0; j < m; ++j) {
    if (kinds[j] < 0 || kinds[j] >= t->n_kinds) return fail(CAMELOT_EINVAL, "kind out of range");
    if (cu[j] < t->cu_step || cu[j] % t->cu_step != 0 || cu[j] / t->cu_step > t->n_shares)
      return fail(CAMELOT_EINVAL, "share out of range");
    if (bi[j] < 0 || bi[j] >= t->n_batches) return fail(CAMELOT_EINVAL, "batch index out of range");
  }
  for (int j = 0; j < m; ++j) feature_row(t, m, kinds, cu, bi, j, feat + (int64_t)j * CAMELOT_PRED_FEATURES);
  return CAMELOT_OK;
}

extern "C" int32_t camelot_predictor_fit_norm(const float* x, int32_t n, float* mean, float* std) {
  clear_error();
  if (!x || n < 1 || !mean || !std) return fail(CAMELOT_EINVAL, "bad normalisation arguments");
  for (int c = 0; c < CAMELOT_PRED_FEATURES; ++c) {
    double s = 0, s2 = 0;
    for (int i = 0; i < n; ++i) s += x[(int64_t)i * CAMELOT_PRED_FEATURES + c];
    const double mu = s / n;
    for (int i = 0; i < n; ++i) {
      const double d = x[(int64_t)i * CAMELOT_PRED_FEATURES + c] - mu;
      s2 += d * d;
    }
    mean[c] = (float)mu;
    std[c] = (float)std::max(std::sqrt(s2 / n), 1e-6);
  }
  return CAMELOT_OK;
}

extern "C" int32_t camelot_predictor_standardize(float* x, int32_t n, const float* mean, const float* std) {
  clear_error();
  if (!x || n < 0 || !mean || !std) return fail(CAMELOT_EINVAL, "bad normalisation arguments");
  for (int i = 0; i < n; ++i)
    for (int c = 0; c < CAMELOT_PRED_FEATURES; ++c) {
      float& v = x[(int64_t)i * CAMELOT_PRED_FEATURES + c];
      v = (v - mean[c]) / std[c];
    }
  return CAMELOT_OK;
}

// ------------------------------------------------------------------ learned allocator
namespace {
typedef __int128 i128;
struct Cand {
  int bi;
  int n[3];
  int k[3];
};
inline int cmp_rat(int64_t an, int64_t ad, int64_t bn, int64_t bd) {
  const i128 l = (i128)an * bd, r = (i128)bn * ad;
  return l < r ? -1 : (l > r ? 1 : 0);
}

// Candidates in lexicographic order (batch index, N_1, k_1, N_2, k_2, ...) that fit
// the CUs, the instance caps and the measured solo table.
void enumerate(const camelot_problem* p, int S, int K, const int* nmax, int total_inst, int bi, int s, int cu_used,
               int inst, Cand& c, std::vector<Cand>& out) {
  if (s == S) {
    out.push_back(c);
    return;
  }
  for (int nn = 1; nn <= nmax[s] && inst + nn <= total_inst; ++nn) {
    for (int kk = 0; kk < K; ++kk) {
      const int cu2 = cu_used + nn * (kk + 1) * p->cu_step;
      if (cu2 > p->cu_total) break;
      if (p->lat_ns[((int64_t)s * K + kk) * p->n_batches + bi] <= 0) continue;
      c.n[s] = nn;
      c.k[s] = kk;
      enumerate(p, S, K, nmax, total_inst, bi, s + 1, cu2, inst + nn, c, out);
    }
  }
}
}  // namespace

namespace {
// Predicts the log co-location slowdown of n feature rows x [n][16] into y [n].
struct SlowdownPredictor {
  virtual ~SlowdownPredictor() = default;
  virtual int32_t predict(float* x, int32_t n, float* y) = 0;
};

// The learned network on the GPU (standardised features).
struct NetPredictor : SlowdownPredictor {
  const float *params, *mean, *std;
  float *dx = nullptr, *dy = nullptr;
  int64_t cap = 0;
  ~NetPredictor() override {
    dfree(dx);
    dfree(dy);
  }
  int32_t predict(float* x, int32_t n, float* y) override {
    int32_t rc = 0;
    if (n > cap) {
      dfree(dx);
      dfree(dy);
      dx = dy = nullptr;
      cap = 0;
      if ((rc = dmalloc(&dx, (size_t)n * CAMELOT_PRED_FEATURES * sizeof(float))) ||
          (rc = dmalloc(&dy, (size_t)n * sizeof(float))))
        return rc;
      cap = n;
    }
    camelot_predictor_standardize(x, n, mean, std);
    if ((rc = h2d(dx, x, (size_t)n * CAMELOT_PRED_FEATURES * sizeof(float)))) return rc;
    hipStream_t s = mem_stream();
    hipLaunchKernelGGL(camelot_pred_forward, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, params,
                       (const float*)dx, (int)n, dy);
    if (hipGetLastError() != hipSuccess) return fail(CAMELOT_EDEVICE, "predictor forward launch failed");
    return d2h(y, dy, (size_t)n * sizeof(float));
  }
};

// A regression tree on the host (raw features).
struct TreePredictor : SlowdownPredictor {
  const camelot_dt* dt;
  int32_t predict(float* x, int32_t n, float* y) override { return camelot_dt_predict(dt, x, n, y); }
};

int32_t alloc_peak_predicted(const camelot_problem* p, const camelot_solo_tables* t, SlowdownPredictor& pred,
                             camelot_alloc* out, int64_t* lat_pred_ns) {
  int32_t rc = check_tables(t);
  if (rc) return rc;
  const int S = p->n_stages;
  if (S < 1 || S > 3 || t->n_kinds != S) return fail(CAMELOT_EINVAL, "learned allocation needs 1..3 stages matching the tables");
  if (p->cu_step != t->cu_step || p->cu_total / p->cu_step > t->n_shares || p->n_batches != t->n_batches)
    return fail(CAMELOT_EINVAL, "solo tables do not cover the problem's shares and batches");
  if (!p->lat_ns || !p->bw_bps || !p->mem_bytes || !p->batches) return fail(CAMELOT_EINVAL, "incomplete problem");
  if (p->max_instances < 1 || p->max_inst_per_stage < 1) return fail(CAMELOT_EINVAL, "instance caps must be >= 1");
  if (p->inst_max)
    for (int i = 0; i < S; ++i)
      if (p->inst_max[i] < 1) return fail(CAMELOT_EINVAL, "inst_max[%d] must be >= 1", i);
  const int K = p->cu_total / p->cu_step;
  int nmax[3];
  const int cap = std::min(p->max_inst_per_stage, p->max_instances);
  for (int i = 0; i < S; ++i) nmax[i] = std::min(cap, p->inst_max ? p->inst_max[i] : cap);
  const int total_inst = std::min(p->max_instances, CAMELOT_MAX_CORUN);
  std::vector<Cand> cands;
  for (int bi = 0; bi < p->n_batches; ++bi) {
    const int64_t wait = p->batch_wait_ns ? p->batch_wait_ns[bi] : 0;
    if (wait > p->qos_ns) continue;
    Cand c{bi, {1, 1, 1}, {0, 0, 0}};
    enumerate(p, S, K, nmax, total_inst, bi, 0, 0, 0, c, cands);
  }
  if (cands.empty()) return fail(CAMELOT_EINFEASIBLE, "no candidate allocation");
  // The predictor gives the log of the co-location slowdown over the solo latency,
  // clamped to [0, 10]: a co-runner never makes a stage faster than it runs alone.
  // So a candidate's solo-table throughput bounds its predicted one from above and
  // its solo latency sum bounds its predicted one from below. Candidates that break
  // a constraint the prediction cannot change (CUs, instances, bandwidth, memory,
  // the QoS already at solo latencies) are dropped; the rest are predicted in
  // chunks in decreasing order of the bound, until the best predicted throughput
  // exceeds the bound of every candidate left. The result is the one a search over
  // every candidate gives: most throughput, then fewest CUs, then least latency,
  // then the first candidate in enumeration order.
  struct Live {
    int64_t tn, td;    // solo-table throughput bound, queries/s = tn / td
    int64_t idx;       // enumeration order
  };
  std::vector<Live> live;
  live.reserve(cands.size());
  for (size_t c = 0; c < cands.size(); ++c) {
    const Cand& cd = cands[c];
    const int bi = cd.bi;
    const int64_t b = p->batches[bi];
    int64_t cu = 0, inst = 0, bw = 0, mem = 0, lat = p->batch_wait_ns ? p->batch_wait_ns[bi] : 0;
    int64_t tn = 0, td = 1;
    for (int s = 0; s < S; ++s) {
      const int kk = cd.k[s], nn = cd.n[s];
      const int64_t Ls = p->lat_ns[((int64_t)s * K + kk) * p->n_batches + bi];
      cu += (int64_t)nn * (kk + 1) * p->cu_step;
      inst += nn;
      bw += nn * p->bw_bps[((int64_t)s * K + kk) * p->n_batches + bi];
      mem += nn * p->mem_bytes[(int64_t)s * p->n_batches + bi];
      lat += Ls;
      const int64_t n1 = (int64_t)nn * b * 1000000000LL;
      if (s == 0 || cmp_rat(n1, Ls, tn, td) < 0) { tn = n1; td = Ls; }
    }
    if (cu > p->cu_total || inst > p->max_instances || bw > p->hbm_bw_budget || mem > p->hbm_bytes_budget ||
        lat > p->qos_ns)
      continue;
    live.push_back({tn, td, (int64_t)c});
  }
  if (live.empty()) return fail(CAMELOT_EINFEASIBLE, "no allocation satisfies the constraints");
  std::stable_sort(live.begin(), live.end(),
                   [](const Live& x, const Live& y) { return cmp_rat(x.tn, x.td, y.tn, y.td) > 0; });
  constexpr int64_t kChunk = 4096;
  std::vector<float> x((size_t)kChunk * S * CAMELOT_PRED_FEATURES), yhat((size_t)kChunk * S);
  bool have = false;
  camelot_alloc best;
  int64_t best_idx = 0;
  int64_t best_lat[3] = {0, 0, 0};
  for (int64_t c0 = 0; c0 < (int64_t)live.size(); c0 += kChunk) {
    // nothing left can reach the best predicted throughput
    if (have && cmp_rat(live[c0].tn, live[c0].td, best.thr_num, best.thr_den) < 0) break;
    const int64_t nc = std::min<int64_t>(kChunk, (int64_t)live.size() - c0);
    for (int64_t c = 0; c < nc; ++c) {
      const Cand& cd = cands[live[c0 + c].idx];
      int32_t kinds[CAMELOT_MAX_CORUN], cu[CAMELOT_MAX_CORUN], bis[CAMELOT_MAX_CORUN], first[3];
      int m = 0;
      for (int s = 0; s < S; ++s) {
        first[s] = m;
        for (int q = 0; q < cd.n[s]; ++q) {
          kinds[m] = s;
          cu[m] = (cd.k[s] + 1) * p->cu_step;
          bis[m] = cd.bi;
          ++m;
        }
      }
      for (int s = 0; s < S; ++s)
        feature_row(t, m, kinds, cu, bis, first[s], x.data() + (c * S + s) * CAMELOT_PRED_FEATURES);
    }
    if ((rc = pred.predict(x.data(), (int32_t)(nc * S), yhat.data()))) return rc;
    for (int64_t c = 0; c < nc; ++c) {
      const int64_t idx = live[c0 + c].idx;
      const Cand& cd = cands[idx];
      const int bi = cd.bi;
      const int64_t b = p->batches[bi];
      int64_t L[3];
      int64_t cu = 0, lat = p->batch_wait_ns ? p->batch_wait_ns[bi] : 0, tn = 0, td = 1;
      for (int s = 0; s < S; ++s) {
        const double y = std::max(0.0, std::min<double>(yhat[c * S + s], 10.0));
        const double solo = (double)p->lat_ns[((int64_t)s * K + cd.k[s]) * p->n_batches + bi];
        L[s] = std::max<int64_t>(1, (int64_t)std::ceil(solo * std::exp(y)));
        cu += (int64_t)cd.n[s] * (cd.k[s] + 1) * p->cu_step;
        lat += L[s];
        const int64_t n1 = (int64_t)cd.n[s] * b * 1000000000LL;
        if (s == 0 || cmp_rat(n1, L[s], tn, td) < 0) { tn = n1; td = L[s]; }
      }
      if (lat > p->qos_ns) continue;
      bool better = !have;
      if (have) {
        const int c1 = cmp_rat(tn, td, best.thr_num, best.thr_den);
        better = c1 > 0 || (c1 == 0 && (cu < best.cu_used || (cu == best.cu_used && (lat < best.lat_ns ||
                                                                                   (lat == best.lat_ns && idx < best_idx)))));
      }
      if (!better) continue;
      have = true;
      best_idx = idx;
      std::memset(&best, 0, sizeof best);
      best.n_stages = S;
      best.batch = (int32_t)b;
      best.batch_index = bi;
      for (int s = 0; s < S; ++s) {
        best.n[s] = cd.n[s];
        best.cu[s] = (cd.k[s] + 1) * p->cu_step;
        best_lat[s] = L[s];
      }
      const int64_t g = std::gcd(tn, td);
      best.thr_num = tn / g;
      best.thr_den = td / g;
      best.lat_ns = lat;
      best.cu_used = cu;
    }
  }
  if (!have) return fail(CAMELOT_EINFEASIBLE, "no allocation satisfies the constraints");
  *out = best;
  if (lat_pred_ns)
    for (int s = 0; s < S; ++s) lat_pred_ns[s] = best_lat[s];
  return CAMELOT_OK;
}
}  // namespace

extern "C" int32_t camelot_alloc_peak_learned(const camelot_problem* p, const camelot_solo_tables* t,
                                              const float* params, const float* mean, const float* std,
                                              camelot_alloc* out, int64_t* lat_pred_ns) {
  clear_error();
  if (!p || !params || !mean || !std || !out) return fail(CAMELOT_EINVAL, "bad learned allocation arguments");
  NetPredictor net;
  net.params = params;
  net.mean = mean;
  net.std = std;
  return alloc_peak_predicted(p, t, net, out, lat_pred_ns);
}

extern "C" int32_t camelot_alloc_peak_dt(const camelot_problem* p, const camelot_solo_tables* t, const camelot_dt* dt,
                                         camelot_alloc* out, int64_t* lat_pred_ns) {
  clear_error();
  if (!p || !dt || !out) return fail(CAMELOT_EINVAL, "bad tree allocation arguments");
  TreePredictor tree;
  tree.dt = dt;
  return alloc_peak_predicted(p, t, tree, out, lat_pred_ns);
}
