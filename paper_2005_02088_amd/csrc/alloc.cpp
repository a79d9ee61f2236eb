// Exact solver of the allocation problems of Section VII over an integer profile
// table: Eq. 1 (maximise the pipeline throughput under the QoS target and the
// resource constraints) and Eq. 3 (minimise the computational resources while the
// throughput reaches a given load).
//
// Search: depth-first over (batch index, N_1, k_1, N_2, k_2, ...) in lexicographic
// order with pruning on the additive constraints (CUs, instances, bandwidth,
// memory, latency are sums of non-negative terms) and on the objective bound
// (the throughput of a partial assignment can only fall as stages are added).
// A candidate replaces the incumbent only when strictly better, so among equal
// candidates the lexicographically first one is kept. Throughputs are compared
// as exact rationals with 128-bit cross products.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>

#include "../../include/camelot.h"
#include "errors.h"

namespace {

constexpr int64_t kNsPerS = 1000000000LL;
typedef __int128 i128;

struct Rat {
  int64_t num = 0, den = 1;   // den > 0
};

inline int cmp(const Rat& a, const Rat& b) {   // sign of a - b
  const i128 l = (i128)a.num * b.den, r = (i128)b.num * a.den;
  return l < r ? -1 : (l > r ? 1 : 0);
}

struct Search {
  const camelot_problem* p;
  int S, K, nmax, bi;
  int nmax_s[CAMELOT_MAX_STAGES];
  int64_t b, wait;
  bool peak;                  // true: Eq. 1; false: Eq. 3 with load
  Rat load;
  int n[CAMELOT_MAX_STAGES], k[CAMELOT_MAX_STAGES];
  bool have = false;
  camelot_alloc best;
  Rat best_thr;

  int64_t lat(int s, int kk) const { return p->lat_ns[((int64_t)s * K + kk) * p->n_batches + bi]; }
  int64_t bw(int s, int kk) const { return p->bw_bps[((int64_t)s * K + kk) * p->n_batches + bi]; }
  int64_t mem(int s) const { return p->mem_bytes[(int64_t)s * p->n_batches + bi]; }

  // true when (thr, cu, lat) is strictly better than the incumbent
  bool better(const Rat& thr, int64_t cu, int64_t latency) const {
    if (!have) return true;
    if (peak) {
      const int c = cmp(thr, best_thr);
      if (c != 0) return c > 0;
      if (cu != best.cu_used) return cu < best.cu_used;
      return latency < best.lat_ns;
    }
    if (cu != best.cu_used) return cu < best.cu_used;
    const int c = cmp(thr, best_thr);
    if (c != 0) return c > 0;
    return latency < best.lat_ns;
  }

  void leaf(const Rat& thr, int64_t cu, int64_t latency) {
    if (!peak && cmp(thr, load) < 0) return;
    if (!better(thr, cu, latency)) return;
    have = true;
    best_thr = thr;
    std::memset(&best, 0, sizeof(best));
    best.n_stages = S;
    best.batch = (int32_t)b;
    best.batch_index = bi;
    for (int s = 0; s < S; ++s) { best.n[s] = n[s]; best.cu[s] = (k[s] + 1) * p->cu_step; }
    const int64_t g = std::gcd(thr.num, thr.den);
    best.thr_num = thr.num / g;
    best.thr_den = thr.den / g;
    best.lat_ns = latency;
    best.cu_used = cu;
  }

  void rec(int s, int64_t cu, int64_t inst, int64_t bwsum, int64_t memsum, int64_t latsum,
           bool has_thr, Rat thr) {
    if (s == S) { leaf(thr, cu, latsum); return; }
    for (int nn = 1; nn <= nmax_s[s]; ++nn) {
      const int64_t inst2 = inst + nn;
      if (inst2 > p->max_instances) break;
      const int64_t mem2 = memsum + nn * mem(s);
      if (mem2 > p->hbm_bytes_budget) break;
      for (int kk = 0; kk < K; ++kk) {
        const int64_t L = lat(s, kk);
        if (L <= 0) continue;
        const int64_t cu2 = cu + (int64_t)nn * (kk + 1) * p->cu_step;
        if (cu2 > p->cu_total) break;                     // shares only grow with kk
        const int64_t bw2 = bwsum + nn * bw(s, kk);
        if (bw2 > p->hbm_bw_budget) continue;
        const int64_t lat2 = latsum + L;
        if (lat2 > p->qos_ns) continue;
        Rat t{(int64_t)nn * b * kNsPerS, L};
        Rat thr2 = (!has_thr || cmp(t, thr) < 0) ? t : thr;
        if (have) {
          if (peak) {
            const int c = cmp(thr2, best_thr);
            if (c < 0) continue;
            if (c == 0 && cu2 > best.cu_used) continue;
          } else {
            if (cu2 > best.cu_used) break;                // larger shares cost more CUs
          }
        }
        if (!peak && cmp(thr2, load) < 0) continue;
        n[s] = nn;
        k[s] = kk;
        rec(s + 1, cu2, inst2, bw2, mem2, lat2, true, thr2);
      }
    }
  }
};

int validate(const camelot_problem* p) {
  if (!p) return camelot::fail(CAMELOT_EINVAL, "problem is NULL");
  if (p->n_stages < 1 || p->n_stages > CAMELOT_MAX_STAGES)
    return camelot::fail(CAMELOT_EINVAL, "n_stages must be in 1..%d", CAMELOT_MAX_STAGES);
  if (p->cu_total < 1 || p->cu_step < 1 || p->cu_total % p->cu_step != 0)
    return camelot::fail(CAMELOT_EINVAL, "cu_total must be a positive multiple of cu_step");
  if (p->max_instances < 1 || p->max_inst_per_stage < 1)
    return camelot::fail(CAMELOT_EINVAL, "instance caps must be >= 1");
  if (p->inst_max)
    for (int i = 0; i < p->n_stages; ++i)
      if (p->inst_max[i] < 1) return camelot::fail(CAMELOT_EINVAL, "inst_max[%d] must be >= 1", i);
  if (p->n_batches < 1 || !p->batches)
    return camelot::fail(CAMELOT_EINVAL, "need at least one batch size");
  for (int j = 0; j < p->n_batches; ++j)
    if (p->batches[j] < 1 || p->batches[j] > (1 << 20))
      return camelot::fail(CAMELOT_EINVAL, "batch sizes must be in 1..2^20");
  if (p->max_inst_per_stage > 1024 || p->max_instances > (1 << 20))
    return camelot::fail(CAMELOT_EINVAL, "instance caps too large");
  if (!p->lat_ns || !p->bw_bps || !p->mem_bytes)
    return camelot::fail(CAMELOT_EINVAL, "lat_ns, bw_bps and mem_bytes are required");
  const int64_t K = p->cu_total / p->cu_step;
  for (int64_t i = 0; i < (int64_t)p->n_stages * K * p->n_batches; ++i)
    if (p->bw_bps[i] < 0) return camelot::fail(CAMELOT_EINVAL, "bw_bps entries must be >= 0");
  for (int64_t i = 0; i < (int64_t)p->n_stages * p->n_batches; ++i)
    if (p->mem_bytes[i] < 0) return camelot::fail(CAMELOT_EINVAL, "mem_bytes entries must be >= 0");
  return CAMELOT_OK;
}

int solve(const camelot_problem* p, bool peak, int64_t load_num, int64_t load_den, camelot_alloc* out) {
  int rc = validate(p);
  if (rc) return rc;
  if (!out) return camelot::fail(CAMELOT_EINVAL, "out is NULL");
  if (!peak && (load_num < 0 || load_den <= 0))
    return camelot::fail(CAMELOT_EINVAL, "load must be a non-negative rational with den > 0");
  Search s;
  s.p = p;
  s.S = p->n_stages;
  s.K = p->cu_total / p->cu_step;
  s.nmax = std::min(p->max_inst_per_stage, p->max_instances);
  for (int i = 0; i < s.S; ++i) s.nmax_s[i] = p->inst_max ? std::min(s.nmax, p->inst_max[i]) : s.nmax;
  s.peak = peak;
  s.load = Rat{load_num, load_den};
  for (int bi = 0; bi < p->n_batches; ++bi) {
    s.bi = bi;
    s.b = p->batches[bi];
    s.wait = p->batch_wait_ns ? p->batch_wait_ns[bi] : 0;
    if (s.wait > p->qos_ns) continue;
    s.rec(0, 0, 0, 0, 0, s.wait, false, Rat{});
  }
  if (!s.have) return camelot::fail(CAMELOT_EINFEASIBLE, "no allocation satisfies the constraints");
  *out = s.best;
  return CAMELOT_OK;
}

// ---------------------------------------------------------------- simulated annealing
// Section VII-C's solver: a state V = (batch index, N_1..N_S, share index k_1..k_S)
// moves one coordinate by +-1 per iteration (coordinate and direction uniform; a
// move off the grid is no move). From a valid state an invalid candidate is
// rejected; a better or equal candidate is taken; a worse one with probability
// exp(-d / temp), d its relative loss (Eq. 1: (T - T') / T; Eq. 3: (R' - R) / R, R the
// CUs in use); temp starts at 0.3 and is multiplied by 0.95 every 100 iterations.
// While the state is invalid every move is taken. The best valid state seen is
// kept with camelot_alloc_peak's / camelot_alloc_min's tie rules (lexicographic
// order of (batch index, N_1, k_1, N_2, k_2, ...) last). Start: the largest batch,
// N_i = 1, k_i = K / S - 1. Random draws: one SplitMix64 stream seeded with `seed`:
// the coordinate (draw mod 2S + 1), the direction (low bit of the next draw), and,
// only when a worse valid candidate is tested, u = (draw >> 11) / 2^53.
constexpr double kSaT0 = 0.3, kSaCooling = 0.95;
constexpr int kSaLevel = 100;

struct SaState {
  int bi;
  int n[CAMELOT_MAX_STAGES], k[CAMELOT_MAX_STAGES];
};

struct SaEval {
  bool ok = false;
  Rat thr;
  int64_t cu = 0, lat = 0;
};

uint64_t sa_next(uint64_t& st) {
  st += 0x9E3779B97F4A7C15ull;
  uint64_t z = st;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

SaEval sa_eval(const camelot_problem* p, int K, const SaState& v, bool peak, const Rat& load) {
  SaEval e;
  const int bi = v.bi;
  const int64_t b = p->batches[bi];
  int64_t inst = 0, bw = 0, mem = 0;
  e.lat = p->batch_wait_ns ? p->batch_wait_ns[bi] : 0;
  bool has = false;
  for (int s = 0; s < p->n_stages; ++s) {
    const int64_t L = p->lat_ns[((int64_t)s * K + v.k[s]) * p->n_batches + bi];
    if (L <= 0) return e;
    e.cu += (int64_t)v.n[s] * (v.k[s] + 1) * p->cu_step;
    inst += v.n[s];
    bw += v.n[s] * p->bw_bps[((int64_t)s * K + v.k[s]) * p->n_batches + bi];
    mem += v.n[s] * p->mem_bytes[(int64_t)s * p->n_batches + bi];
    e.lat += L;
    const Rat t{(int64_t)v.n[s] * b * kNsPerS, L};
    if (!has || cmp(t, e.thr) < 0) e.thr = t;
    has = true;
  }
  if (e.cu > p->cu_total || inst > p->max_instances || bw > p->hbm_bw_budget || mem > p->hbm_bytes_budget ||
      e.lat > p->qos_ns)
    return e;
  if (!peak && cmp(e.thr, load) < 0) return e;
  e.ok = true;
  return e;
}

// true when (a, va) beats (b, vb) under the exhaustive solvers' tie rules
bool sa_better(const SaEval& a, const SaState& va, const SaEval& b, const SaState& vb, int S, bool peak) {
  if (peak) {
    const int c = cmp(a.thr, b.thr);
    if (c != 0) return c > 0;
    if (a.cu != b.cu) return a.cu < b.cu;
  } else {
    if (a.cu != b.cu) return a.cu < b.cu;
    const int c = cmp(a.thr, b.thr);
    if (c != 0) return c > 0;
  }
  if (a.lat != b.lat) return a.lat < b.lat;
  if (va.bi != vb.bi) return va.bi < vb.bi;
  for (int s = 0; s < S; ++s) {
    if (va.n[s] != vb.n[s]) return va.n[s] < vb.n[s];
    if (va.k[s] != vb.k[s]) return va.k[s] < vb.k[s];
  }
  return false;
}

int solve_sa(const camelot_problem* p, bool peak, int64_t load_num, int64_t load_den, int32_t iters, uint64_t seed,
             camelot_alloc* out) {
  int rc = validate(p);
  if (rc) return rc;
  if (!out) return camelot::fail(CAMELOT_EINVAL, "out is NULL");
  if (iters < 0) return camelot::fail(CAMELOT_EINVAL, "iters must be >= 0");
  if (!peak && (load_num < 0 || load_den <= 0))
    return camelot::fail(CAMELOT_EINVAL, "load must be a non-negative rational with den > 0");
  const int S = p->n_stages, K = p->cu_total / p->cu_step, D = 2 * S + 1;
  const Rat load{load_num, load_den};
  int nmax[CAMELOT_MAX_STAGES];
  for (int s = 0; s < S; ++s) {
    nmax[s] = std::min(p->max_inst_per_stage, p->max_instances);
    if (p->inst_max) nmax[s] = std::min(nmax[s], p->inst_max[s]);
  }
  SaState cur;
  std::memset(&cur, 0, sizeof cur);
  cur.bi = p->n_batches - 1;
  for (int s = 0; s < S; ++s) {
    cur.n[s] = 1;
    cur.k[s] = std::max(0, K / S - 1);
  }
  SaEval ecur = sa_eval(p, K, cur, peak, load), ebest = ecur;
  SaState best = cur;
  uint64_t rng = seed;
  double temp = kSaT0;
  for (int32_t t = 0; t < iters; ++t) {
    if (t > 0 && t % kSaLevel == 0) temp *= kSaCooling;
    const int c = (int)(sa_next(rng) % (uint64_t)D);
    const int step = (sa_next(rng) & 1u) ? 1 : -1;
    SaState cand = cur;
    if (c == 0) {
      cand.bi += step;
      if (cand.bi < 0 || cand.bi >= p->n_batches) continue;
    } else if (c <= S) {
      cand.n[c - 1] += step;
      if (cand.n[c - 1] < 1 || cand.n[c - 1] > nmax[c - 1]) continue;
    } else {
      cand.k[c - S - 1] += step;
      if (cand.k[c - S - 1] < 0 || cand.k[c - S - 1] >= K) continue;
    }
    const SaEval ec = sa_eval(p, K, cand, peak, load);
    bool take;
    if (!ecur.ok) {
      take = true;
    } else if (!ec.ok) {
      take = false;
    } else {
      double d;
      if (peak) {
        const double tc = (double)ecur.thr.num / (double)ecur.thr.den, tn = (double)ec.thr.num / (double)ec.thr.den;
        d = (tc - tn) / tc;
      } else {
        d = (double)(ec.cu - ecur.cu) / (double)ecur.cu;
      }
      if (d <= 0) {
        take = true;
      } else {
        const double u = (double)(sa_next(rng) >> 11) / 9007199254740992.0;
        take = u < std::exp(-d / temp);
      }
    }
    if (!take) continue;
    cur = cand;
    ecur = ec;
    if (ecur.ok && (!ebest.ok || sa_better(ecur, cur, ebest, best, S, peak))) {
      ebest = ecur;
      best = cur;
    }
  }
  if (!ebest.ok) return camelot::fail(CAMELOT_EINFEASIBLE, "annealing visited no valid allocation");
  std::memset(out, 0, sizeof *out);
  out->n_stages = S;
  out->batch_index = best.bi;
  out->batch = p->batches[best.bi];
  for (int s = 0; s < S; ++s) {
    out->n[s] = best.n[s];
    out->cu[s] = (best.k[s] + 1) * p->cu_step;
  }
  const int64_t g = std::gcd(ebest.thr.num, ebest.thr.den);
  out->thr_num = ebest.thr.num / g;
  out->thr_den = ebest.thr.den / g;
  out->lat_ns = ebest.lat;
  out->cu_used = ebest.cu;
  return CAMELOT_OK;
}

}  // namespace

extern "C" int32_t camelot_alloc_peak(const camelot_problem* problem, camelot_alloc* out) {
  camelot::clear_error();
  return solve(problem, true, 0, 1, out);
}

extern "C" int32_t camelot_alloc_min(const camelot_problem* problem, int64_t load_num, int64_t load_den,
                                     camelot_alloc* out) {
  camelot::clear_error();
  return solve(problem, false, load_num, load_den, out);
}

extern "C" int32_t camelot_alloc_eval(const camelot_problem* p, camelot_alloc* a) {
  camelot::clear_error();
  int rc = validate(p);
  if (rc) return rc;
  if (!a) return camelot::fail(CAMELOT_EINVAL, "alloc is NULL");
  const int K = p->cu_total / p->cu_step;
  const int bi = a->batch_index;
  if (bi < 0 || bi >= p->n_batches) return camelot::fail(CAMELOT_EINVAL, "batch_index out of range");
  const int64_t b = p->batches[bi];
  int64_t cu = 0, inst = 0, bw = 0, mem = 0;
  int64_t lat = p->batch_wait_ns ? p->batch_wait_ns[bi] : 0;
  Rat thr{0, 1};
  bool has = false;
  for (int s = 0; s < p->n_stages; ++s) {
    const int nn = a->n[s];
    if (nn < 1 || a->cu[s] < p->cu_step || a->cu[s] % p->cu_step != 0 || a->cu[s] > p->cu_total)
      return camelot::fail(CAMELOT_EINVAL, "stage %d: bad instance count or share", s);
    const int kk = a->cu[s] / p->cu_step - 1;
    const int64_t L = p->lat_ns[((int64_t)s * K + kk) * p->n_batches + bi];
    if (L <= 0) return camelot::fail(CAMELOT_EINFEASIBLE, "stage %d: unmeasured table point", s);
    cu += (int64_t)nn * a->cu[s];
    inst += nn;
    bw += nn * p->bw_bps[((int64_t)s * K + kk) * p->n_batches + bi];
    mem += nn * p->mem_bytes[(int64_t)s * p->n_batches + bi];
    lat += L;
    Rat t{(int64_t)nn * b * kNsPerS, L};
    if (!has || cmp(t, thr) < 0) thr = t;
    has = true;
  }
  a->n_stages = p->n_stages;
  a->batch = (int32_t)b;
  const int64_t g = std::gcd(thr.num, thr.den);
  a->thr_num = thr.num / g;
  a->thr_den = thr.den / g;
  a->lat_ns = lat;
  a->cu_used = cu;
  if (cu > p->cu_total || inst > p->max_instances || bw > p->hbm_bw_budget ||
      mem > p->hbm_bytes_budget || lat > p->qos_ns)
    return camelot::fail(CAMELOT_EINFEASIBLE, "allocation violates a constraint");
  return CAMELOT_OK;
}

extern "C" int32_t camelot_alloc_sa(const camelot_problem* problem, int32_t objective, int64_t load_num,
                                    int64_t load_den, int32_t iters, uint64_t seed, camelot_alloc* out) {
  camelot::clear_error();
  if (objective != CAMELOT_OBJ_PEAK && objective != CAMELOT_OBJ_MIN)
    return camelot::fail(CAMELOT_EINVAL, "objective must be CAMELOT_OBJ_PEAK or CAMELOT_OBJ_MIN");
  return solve_sa(problem, objective == CAMELOT_OBJ_PEAK, load_num, load_den, iters, seed, out);
}
