// Decision-tree regressor: the kind of latency predictor the paper trains on its
// co-location profiles (Section VII-A), here beside the learned MLP predictor.
// CART regression (Breiman et al., 1984) with the squared error: a node holding
// samples S splits on the feature and threshold that maximise
//   sum_L^2 / n_L + sum_R^2 / n_R
// (equivalently, that minimise the children's summed squared error), over the
// midpoints between consecutive distinct values of each feature, both children
// keeping at least min_leaf samples; it becomes a leaf (value = mean of y over S)
// at max_depth, when it cannot be split so, or when no split lowers the error.
// Deterministic: features in index order, samples of a feature in (value, index)
// order, sums accumulated in that order in double, the first best split kept.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "../../include/camelot.h"
#include "errors.h"

struct camelot_dt {
  std::vector<int32_t> feat;     // split feature, -1 for a leaf
  std::vector<double> thr;       // x[feat] <= thr goes left
  std::vector<double> value;     // mean of y over the node's samples
  std::vector<int32_t> left, right;
  int32_t n_feat = 0;
};

namespace camelot {
namespace {

struct Fit {
  const float* x;
  const float* y;
  int32_t n_feat;
  int32_t max_depth;
  int32_t min_leaf;
  camelot_dt* t;
  std::vector<int32_t> order;    // scratch: the node's samples sorted by one feature
};

int32_t new_node(camelot_dt* t, double value) {
  t->feat.push_back(-1);
  t->thr.push_back(0.0);
  t->value.push_back(value);
  t->left.push_back(-1);
  t->right.push_back(-1);
  return (int32_t)t->feat.size() - 1;
}

// Builds the subtree over samples idx (in ascending index order); returns its node.
int32_t grow(Fit& f, const std::vector<int32_t>& idx, int32_t depth) {
  const int32_t n = (int32_t)idx.size();
  double total = 0.0;
  for (int32_t i : idx) total += (double)f.y[i];
  const int32_t node = new_node(f.t, total / (double)n);
  if (depth >= f.max_depth || n < 2 * f.min_leaf) return node;
  const double parent = total * total / (double)n;
  double best = parent;
  int32_t best_f = -1;
  double best_thr = 0.0;
  for (int32_t k = 0; k < f.n_feat; ++k) {
    f.order = idx;
    std::stable_sort(f.order.begin(), f.order.end(), [&](int32_t a, int32_t b) {
      return f.x[(int64_t)a * f.n_feat + k] < f.x[(int64_t)b * f.n_feat + k];
    });
    double sl = 0.0;
    for (int32_t i = 1; i < n; ++i) {
      sl += (double)f.y[f.order[i - 1]];
      if (i < f.min_leaf || n - i < f.min_leaf) continue;
      const float a = f.x[(int64_t)f.order[i - 1] * f.n_feat + k];
      const float b = f.x[(int64_t)f.order[i] * f.n_feat + k];
      if (!(a < b)) continue;
      const double sr = total - sl;
      const double g = sl * sl / (double)i + sr * sr / (double)(n - i);
      if (g > best) {
        best = g;
        best_f = k;
        best_thr = 0.5 * ((double)a + (double)b);
      }
    }
  }
  if (best_f < 0) return node;
  std::vector<int32_t> li, ri;
  for (int32_t i : idx) ((double)f.x[(int64_t)i * f.n_feat + best_f] <= best_thr ? li : ri).push_back(i);
  f.t->feat[node] = best_f;
  f.t->thr[node] = best_thr;
  const int32_t l = grow(f, li, depth + 1);
  f.t->left[node] = l;
  const int32_t r = grow(f, ri, depth + 1);
  f.t->right[node] = r;
  return node;
}

}  // namespace
}  // namespace camelot

using camelot::fail;

extern "C" int32_t camelot_dt_fit(const float* x, const float* y, int32_t n, int32_t n_feat, int32_t max_depth,
                                  int32_t min_leaf, camelot_dt** out) {
  camelot::clear_error();
  if (!out) return fail(CAMELOT_EINVAL, "out is NULL");
  *out = nullptr;
  if (!x || !y) return fail(CAMELOT_EINVAL, "x/y are NULL");
  if (n < 1 || n_feat < 1 || max_depth < 0 || max_depth > 64 || min_leaf < 1)
    return fail(CAMELOT_EINVAL, "need n >= 1, n_feat >= 1, 0 <= max_depth <= 64, min_leaf >= 1");
  for (int64_t i = 0; i < (int64_t)n * n_feat; ++i)
    if (!std::isfinite(x[i])) return fail(CAMELOT_EINVAL, "x[%lld] is not finite", (long long)i);
  for (int32_t i = 0; i < n; ++i)
    if (!std::isfinite(y[i])) return fail(CAMELOT_EINVAL, "y[%d] is not finite", i);
  camelot_dt* t = new (std::nothrow) camelot_dt;
  if (!t) return fail(CAMELOT_ENOMEM, "out of host memory");
  t->n_feat = n_feat;
  camelot::Fit f{x, y, n_feat, max_depth, min_leaf, t, {}};
  std::vector<int32_t> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  try {
    camelot::grow(f, idx, 0);
  } catch (const std::bad_alloc&) {
    delete t;
    return fail(CAMELOT_ENOMEM, "out of host memory");
  }
  *out = t;
  return CAMELOT_OK;
}

extern "C" int32_t camelot_dt_predict(const camelot_dt* t, const float* x, int32_t n, float* out) {
  camelot::clear_error();
  if (!t || (n > 0 && (!x || !out))) return fail(CAMELOT_EINVAL, "tree/x/out are NULL");
  if (n < 0) return fail(CAMELOT_EINVAL, "n must be >= 0");
  for (int32_t i = 0; i < n; ++i) {
    const float* r = x + (int64_t)i * t->n_feat;
    int32_t k = 0;
    while (t->feat[k] >= 0) k = (double)r[t->feat[k]] <= t->thr[k] ? t->left[k] : t->right[k];
    out[i] = (float)t->value[k];
  }
  return CAMELOT_OK;
}

extern "C" int32_t camelot_dt_export(const camelot_dt* t, int32_t cap, int32_t* n_nodes, int32_t* feat, double* thr,
                                     double* value, int32_t* left, int32_t* right) {
  camelot::clear_error();
  if (!t || !n_nodes) return fail(CAMELOT_EINVAL, "tree/n_nodes are NULL");
  const int32_t m = (int32_t)t->feat.size();
  *n_nodes = m;
  if (cap <= 0) return CAMELOT_OK;
  if (cap < m) return fail(CAMELOT_EINVAL, "cap %d < %d nodes", cap, m);
  if (!feat || !thr || !value || !left || !right) return fail(CAMELOT_EINVAL, "output arrays are NULL");
  std::memcpy(feat, t->feat.data(), sizeof(int32_t) * m);
  std::memcpy(thr, t->thr.data(), sizeof(double) * m);
  std::memcpy(value, t->value.data(), sizeof(double) * m);
  std::memcpy(left, t->left.data(), sizeof(int32_t) * m);
  std::memcpy(right, t->right.data(), sizeof(int32_t) * m);
  return CAMELOT_OK;
}

extern "C" void camelot_dt_destroy(camelot_dt* t) { delete t; }
