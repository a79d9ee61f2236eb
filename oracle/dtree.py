"""Decision-tree regressor, plain NumPy (test infrastructure only).

The paper fits a decision tree to its co-location profiles to predict a stage's
latency under contention (Section VII-A). This is the regression tree of CART
(Breiman, Friedman, Olshen & Stone, 1984) with the squared error, written from that
definition:

* a node holds a set S of samples and predicts the mean of their y;
* it is split on the feature f and threshold t that minimise the summed squared
  error of the two children {x_f <= t} and {x_f > t}, which for fixed S is the same
  as maximising  sum_L^2 / n_L + sum_R^2 / n_R;
* candidate thresholds are the midpoints between consecutive distinct values of
  x_f over S; both children must keep at least min_leaf samples;
* a node is a leaf at depth max_depth, when no candidate exists, or when the best
  candidate does not lower the error (gain not above sum^2 / n).

Readings where CART leaves a choice (listed in the design notes): features are tried
in index order and the first best split is kept (ties go to the lower feature, then
the lower threshold); samples of a feature are taken in (value, index) order and the
sums are accumulated in that order in float64; the midpoint is computed in float64
from the float32 values. Nodes are numbered in creation order (depth first, left
child first). Nothing here is shared with the library.
"""
import numpy as np


def fit(x, y, max_depth, min_leaf):
    """Returns the tree as dict(feat, thr, value, left, right) of equal-length lists
    (feat -1 and children -1 for a leaf)."""
    x = np.asarray(x, np.float32)
    y = np.asarray(y, np.float32)
    n, n_feat = x.shape
    tree = {"feat": [], "thr": [], "value": [], "left": [], "right": []}

    def new_node(value):
        for k, v in (("feat", -1), ("thr", 0.0), ("value", value), ("left", -1), ("right", -1)):
            tree[k].append(v)
        return len(tree["feat"]) - 1

    def grow(idx, depth):
        m = len(idx)
        ys = y[idx].astype(np.float64)
        total = float(np.cumsum(ys)[-1])
        node = new_node(total / m)
        if depth >= max_depth or m < 2 * min_leaf:
            return node
        best, best_f, best_thr = total * total / m, -1, 0.0
        for f in range(n_feat):
            order = idx[np.argsort(x[idx, f], kind="stable")]
            xs = x[order, f]
            sl_all = np.cumsum(y[order].astype(np.float64))       # sl_all[i - 1] = sum of the first i
            for i in range(1, m):
                if i < min_leaf or m - i < min_leaf or not xs[i - 1] < xs[i]:
                    continue
                sl = sl_all[i - 1]
                sr = total - sl
                g = sl * sl / i + sr * sr / (m - i)
                if g > best:
                    best, best_f, best_thr = g, f, 0.5 * (float(xs[i - 1]) + float(xs[i]))
        if best_f < 0:
            return node
        go_left = x[idx, best_f].astype(np.float64) <= best_thr
        tree["feat"][node] = best_f
        tree["thr"][node] = best_thr
        tree["left"][node] = grow(idx[go_left], depth + 1)
        tree["right"][node] = grow(idx[~go_left], depth + 1)
        return node

    grow(np.arange(n), 0)
    return tree


def predict(tree, x):
    """Predictions (float32) for the rows of x."""
    x = np.asarray(x, np.float32)
    out = np.empty(x.shape[0], np.float32)
    for r in range(x.shape[0]):
        k = 0
        while tree["feat"][k] >= 0:
            k = tree["left"][k] if float(x[r, tree["feat"][k]]) <= tree["thr"][k] else tree["right"][k]
        out[r] = np.float32(tree["value"][k])
    return out


def sse(tree, x, y):
    """Summed squared error of the tree's predictions (float64)."""
    d = predict(tree, x).astype(np.float64) - np.asarray(y, np.float64)
    return float(d @ d)
