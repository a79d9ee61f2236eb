"""Decision-tree latency predictor (CART regression, the paper's predictor kind,
Section VII-A): the oracle against what the definition fixes, then the library's
host implementation against the oracle, node for node and prediction for prediction."""
import numpy as np
import pytest

from oracle import dtree as OD
from paper_2005_02088_amd import camelot as cm
import workload_gen as G


def _leaves(tree):
    return [k for k, f in enumerate(tree["feat"]) if f < 0]


def _leaf_of(tree, row):
    k = 0
    while tree["feat"][k] >= 0:
        k = tree["left"][k] if float(row[tree["feat"][k]]) <= tree["thr"][k] else tree["right"][k]
    return k


# ---------------------------------------------------------------- oracle pins
def test_oracle_depth_zero_is_the_mean():
    g = G.rng("dtree", 1)
    x = g.standard_normal((40, 3)).astype(np.float32)
    y = g.standard_normal(40).astype(np.float32)
    t = OD.fit(x, y, max_depth=0, min_leaf=1)
    assert t["feat"] == [-1]
    assert t["value"][0] == pytest.approx(float(np.mean(y.astype(np.float64))), rel=1e-12)


def test_oracle_recovers_a_step_exactly():
    g = G.rng("dtree", 2)
    x = g.uniform(0, 1, (200, 2)).astype(np.float32)
    y = np.where(x[:, 1] > 0.3, 2.0, -1.0).astype(np.float32)
    t = OD.fit(x, y, max_depth=3, min_leaf=1)
    # one split on feature 1 between the two samples around 0.3, two pure leaves
    assert t["feat"][0] == 1 and len(t["feat"]) == 3
    lo = float(x[x[:, 1] <= 0.3, 1].max())
    hi = float(x[x[:, 1] > 0.3, 1].min())
    assert t["thr"][0] == 0.5 * (lo + hi)
    assert np.array_equal(OD.predict(t, x), y)


def test_oracle_recovers_a_two_level_staircase():
    """y = 2 [x0 > 0.5] + [x1 > 0.6]: the root splits x0 (the larger step), each child
    then splits x1, and depth 2 reproduces y exactly (4 pure leaves)."""
    g = G.rng("dtree", 5)
    x = g.uniform(0, 1, (300, 3)).astype(np.float32)
    y = (2.0 * (x[:, 0] > 0.5) + 1.0 * (x[:, 1] > 0.6)).astype(np.float32)
    t = OD.fit(x, y, max_depth=2, min_leaf=1)
    assert t["feat"][0] == 0
    assert len(_leaves(t)) == 4
    assert np.array_equal(OD.predict(t, x), y)


def test_oracle_first_split_is_the_brute_force_best():
    """Depth 1: the oracle's split has the least summed squared error over every
    (feature, threshold between distinct values) with both sides >= min_leaf,
    computed from the two subsets directly."""
    g = G.rng("dtree", 3)
    for trial in range(5):
        x = np.round(g.uniform(0, 4, (23, 3)), 1).astype(np.float32)    # ties on purpose
        y = g.standard_normal(23).astype(np.float32)
        min_leaf = 1 + trial % 3
        t = OD.fit(x, y, max_depth=1, min_leaf=min_leaf)
        yd = y.astype(np.float64)

        def sse_of(mask):
            a, b = yd[mask], yd[~mask]
            return float(((a - a.mean()) ** 2).sum() + ((b - b.mean()) ** 2).sum())

        best = float(((yd - yd.mean()) ** 2).sum())
        for f in range(3):
            vals = np.unique(x[:, f])
            for lo, hi in zip(vals[:-1], vals[1:]):
                mask = x[:, f] <= 0.5 * (float(lo) + float(hi))
                if mask.sum() >= min_leaf and (~mask).sum() >= min_leaf:
                    best = min(best, sse_of(mask))
        if t["feat"][0] < 0:
            assert best == pytest.approx(float(((yd - yd.mean()) ** 2).sum()), rel=1e-12)
        else:
            got = sse_of(x[:, t["feat"][0]].astype(np.float64) <= t["thr"][0])
            assert got == pytest.approx(best, rel=1e-9, abs=1e-12)


def test_oracle_leaves_respect_min_leaf_and_error_falls_with_depth():
    g = G.rng("dtree", 4)
    x = g.standard_normal((300, 4)).astype(np.float32)
    y = (np.sin(2 * x[:, 0]) + 0.5 * x[:, 1] * x[:, 2] + 0.1 * g.standard_normal(300)).astype(np.float32)
    prev = None
    for depth in range(0, 7):
        t = OD.fit(x, y, max_depth=depth, min_leaf=7)
        counts = {}
        for row in x:
            k = _leaf_of(t, row)
            counts[k] = counts.get(k, 0) + 1
        assert set(counts) == set(_leaves(t))
        assert min(counts.values()) >= 7
        e = OD.sse(t, x, y)
        if prev is not None:
            assert e <= prev + 1e-9
        prev = e


# ---------------------------------------------------------------- library vs oracle
def _lib_tree(x, y, depth, min_leaf):
    t = cm.camelot_dt_fit(x, y, depth, min_leaf)
    return t, t.export()


@pytest.mark.parametrize("n,n_feat,depth,min_leaf,seed", [
    (1, 3, 4, 1, 0),
    (17, 2, 3, 1, 1),
    (120, 5, 6, 3, 2),
    (400, 16, 8, 10, 3),
])
def test_library_tree_matches_oracle(n, n_feat, depth, min_leaf, seed):
    g = G.rng("dtree", 10 + seed)
    x = g.standard_normal((n, n_feat)).astype(np.float32)
    if n > 1:
        x[:, 0] = np.round(x[:, 0], 1)             # ties in one feature
    y = (x[:, 0] * 1.5 + np.abs(x[:, -1]) + 0.2 * g.standard_normal(n)).astype(np.float32)
    o = OD.fit(x, y, depth, min_leaf)
    t, e = _lib_tree(x, y, depth, min_leaf)
    assert list(e["feat"]) == o["feat"]
    assert list(e["left"]) == o["left"] and list(e["right"]) == o["right"]
    assert np.array_equal(e["thr"], np.array(o["thr"], np.float64))
    assert np.array_equal(e["value"], np.array(o["value"], np.float64))
    xq = g.standard_normal((64, n_feat)).astype(np.float32)
    assert np.array_equal(t.predict(xq).view(np.uint32), OD.predict(o, xq).view(np.uint32))
    assert np.array_equal(t.predict(x).view(np.uint32), OD.predict(o, x).view(np.uint32))


def test_library_rejects_bad_input():
    x = np.zeros((4, 2), np.float32)
    y = np.zeros(4, np.float32)
    for args in ((x, y, -1, 1), (x, y, 3, 0), (x, y, 65, 1)):
        with pytest.raises(cm.CamelotError) as ei:
            cm.camelot_dt_fit(*args)
        assert ei.value.code == cm.EINVAL
    xn = x.copy()
    xn[1, 1] = np.nan
    with pytest.raises(cm.CamelotError):
        cm.camelot_dt_fit(xn, y, 3, 1)


# ---------------------------------------------------------------- the tree as the allocator's predictor
def test_tree_allocator_matches_brute_force():
    """camelot_alloc_peak_dt against a brute force written from Eq. 1: every candidate
    (batch, N_i, share_i) in lexicographic order, each stage's latency its solo
    latency times exp(the oracle tree's prediction from the candidate's co-location
    features), the most throughput, then fewer CUs, then less latency, the first
    candidate on a full tie."""
    import math
    from fractions import Fraction

    g = G.rng("dtree", 30)
    S, step, cu_total, batches = 2, 8, 32, [1, 2, 4]
    K, nb = cu_total // step, len(batches)
    lat = g.integers(5_000, 200_000, (S, K, nb)).astype(np.int64)
    lat[1, 0, 2] = 0                                  # an unmeasured point is skipped
    hbm = g.uniform(0, 1, (S, K, nb)).astype(np.float32)
    mfma = g.uniform(0, 1, (S, K, nb)).astype(np.float32)
    tabs = cm.SoloTablesArrays(step, batches, hbm, mfma)
    prob = cm.ProblemArrays(cu_total=cu_total, cu_step=step, max_instances=4, max_inst_per_stage=3,
                            batches=batches, qos_ns=400_000, hbm_bytes_budget=1 << 62, hbm_bw_budget=1 << 62,
                            lat_ns=lat, bw_bps=np.zeros_like(lat), mem_bytes=np.zeros((S, nb), np.int64),
                            inst_max=[1, 3])
    # a tree fitted to random features -> log slowdowns in [0, 1)
    xt = g.uniform(0, 1, (300, 16)).astype(np.float32)
    yt = g.uniform(0, 1, 300).astype(np.float32)
    tree = cm.camelot_dt_fit(xt, yt, 5, 4)
    otree = OD.fit(xt, yt, 5, 4)

    best = None
    for bi, b in enumerate(batches):
        nmax = [1, 3]
        for n0 in range(1, nmax[0] + 1):
            for k0 in range(K):
                cu0 = n0 * (k0 + 1) * step
                if cu0 > cu_total:
                    break
                if lat[0, k0, bi] <= 0:
                    continue
                for n1 in range(1, nmax[1] + 1):
                    if n0 + n1 > 4:
                        break
                    for k1 in range(K):
                        cu = cu0 + n1 * (k1 + 1) * step
                        if cu > cu_total:
                            break
                        if lat[1, k1, bi] <= 0:
                            continue
                        kinds = [0] * n0 + [1] * n1
                        cus = [(k0 + 1) * step] * n0 + [(k1 + 1) * step] * n1
                        f = cm.camelot_predictor_features(tabs, kinds, cus, [bi] * (n0 + n1))
                        yp = OD.predict(otree, f[[0, n0]])
                        L = []
                        for s, k in ((0, k0), (1, k1)):
                            y = max(0.0, min(float(yp[s]), 10.0))     # co-runners never speed up
                            L.append(max(1, math.ceil(float(lat[s, k, bi]) * math.exp(y))))
                        tot = sum(L)
                        if tot > 400_000:
                            continue
                        thr = min(Fraction(n * b * 10**9, l) for n, l in ((n0, L[0]), (n1, L[1])))
                        key = (thr, -cu, -tot)
                        if best is None or key > best[0]:
                            best = (key, bi, [n0, n1], [(k0 + 1) * step, (k1 + 1) * step], L)
    a, lp = cm.camelot_alloc_peak_dt(prob, tabs, tree)
    assert best is not None and a is not None
    d = a.as_dict()
    assert (d["batch_index"], d["n"][:S], d["cu"][:S]) == (best[1], best[2], best[3])
    assert Fraction(d["thr_num"], d["thr_den"]) == best[0][0]
    assert list(lp) == best[4]


def test_tree_allocator_infeasible_and_predict_empty():
    g = G.rng("dtree", 31)
    S, step, batches = 2, 8, [1, 2]
    lat = g.integers(5_000, 20_000, (S, 4, 2)).astype(np.int64)
    tabs = cm.SoloTablesArrays(step, batches, np.zeros((S, 4, 2), np.float32), np.zeros((S, 4, 2), np.float32))
    tree = cm.camelot_dt_fit(g.uniform(0, 1, (20, 16)).astype(np.float32), np.zeros(20, np.float32), 3, 1)
    prob = cm.ProblemArrays(cu_total=32, cu_step=step, max_instances=2, max_inst_per_stage=1, batches=batches,
                            qos_ns=1_000, hbm_bytes_budget=1 << 62, hbm_bw_budget=1 << 62, lat_ns=lat,
                            bw_bps=np.zeros_like(lat), mem_bytes=np.zeros((S, 2), np.int64))
    a, lp = cm.camelot_alloc_peak_dt(prob, tabs, tree)      # no candidate meets a 1 us QoS
    assert a is None and lp is None
    assert tree.predict(np.zeros((0, 16), np.float32)).shape == (0,)
