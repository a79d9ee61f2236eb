"""The library's allocator (C++, exact search) returns the same allocation as the
oracle's brute force, bit for bit, given the same integer table."""
import numpy as np
import pytest

from oracle import alloc as OA
from paper_2005_02088_amd import camelot as cm
import workload_gen as G

BIG = (1 << 62)


def _both(lat, bw, mem, batches, cu_total, cu_step, *, qos=BIG, nmax=1, I=48, bw_budget=BIG,
          mem_budget=BIG, wait=None, inst_max=None):
    lat = np.asarray(lat, np.int64)
    bw = np.asarray(bw, np.int64)
    mem = np.asarray(mem, np.int64)
    po = OA.Problem(cu_total=cu_total, cu_step=cu_step, max_instances=I, max_inst_per_stage=nmax,
                    batches=list(batches), qos_ns=qos, hbm_bytes_budget=mem_budget, hbm_bw_budget=bw_budget,
                    lat_ns=lat, bw_bps=bw, mem_bytes=mem, batch_wait_ns=wait, inst_max=inst_max)
    pc = cm.ProblemArrays(cu_total=cu_total, cu_step=cu_step, max_instances=I, max_inst_per_stage=nmax,
                          batches=batches, qos_ns=qos, hbm_bytes_budget=mem_budget, hbm_bw_budget=bw_budget,
                          lat_ns=lat, bw_bps=bw, mem_bytes=mem, batch_wait_ns=wait, inst_max=inst_max)
    return po, pc


def _same(o, c):
    if o is None:
        assert c is None
        return
    assert c is not None
    d = c.as_dict()
    assert d["batch"] == o.batch and d["batch_index"] == o.batch_index
    assert d["n"] == o.n and d["cu"] == o.cu
    assert (d["thr_num"], d["thr_den"]) == (o.thr_num, o.thr_den)
    assert d["lat_ns"] == o.lat_ns and d["cu_used"] == o.cu_used


def test_hand_grid():
    lat = [[[1000], [600], [450], [400]], [[500], [400], [350], [330]]]
    z = np.zeros((2, 4, 1), np.int64)
    po, pc = _both(lat, z, np.zeros((2, 1)), [2], 16, 4)
    _same(OA.alloc_peak(po), cm.camelot_alloc_peak(pc))
    for lam in (1_000_000, 3_000_000, 5_000_000):
        _same(OA.alloc_min(po, lam, 1), cm.camelot_alloc_min(pc, lam, 1))


@pytest.mark.parametrize("sub", range(12))
def test_random_tables_match_brute_force(sub):
    g = G.rng("tables", 99, sub)
    S = int(g.integers(1, 4))
    K = int(g.integers(2, 7))
    batches = sorted(set(int(b) for b in g.choice([1, 2, 4, 8, 16, 32], int(g.integers(1, 4)), replace=False)))
    lat, bw, mem = G.random_problem_tables(S, K, batches, seed=7, sub=sub)
    # sprinkle unmeasured points and exact ties
    lat[g.random(lat.shape) < 0.1] = 0
    if lat.shape[1] > 1:
        lat[:, 1, :] = lat[:, 0, :]
    nmax = int(g.integers(1, 3))
    kw = dict(nmax=nmax, I=int(g.integers(S, S * nmax + 1)),
              qos=int(np.sort(lat.reshape(-1))[-1] * S * g.uniform(0.3, 1.2)),
              bw_budget=int(bw.max() * g.uniform(0.8, 3)), mem_budget=int(mem.max() * g.uniform(1, 4)),
              wait=[int(x) for x in g.integers(0, 2000, len(batches))])
    cu_step = 8
    po, pc = _both(lat, bw, mem, batches, K * cu_step, cu_step, **kw)
    o = OA.alloc_peak(po)
    _same(o, cm.camelot_alloc_peak(pc))
    if o is not None:
        for frac in (1, 3, 7, 10):
            num, den = o.thr_num * frac, o.thr_den * 10
            _same(OA.alloc_min(po, num, den), cm.camelot_alloc_min(pc, num, den))
    _same(OA.alloc_min(po, 1, 1), cm.camelot_alloc_min(pc, 1, 1))


def test_speech_sized_grid_matches_brute_force():
    # three stages, 16 shares of 16 CUs, four batch sizes: 16^3 * 4 points
    batches = [1, 8, 32, 128]
    lat, bw, mem = G.random_problem_tables(3, 16, batches, seed=3)
    po, pc = _both(lat, bw, mem, batches, 256, 16, qos=int(lat.max()), bw_budget=int(bw.max() * 2),
                   mem_budget=int(mem.max() * 3))
    _same(OA.alloc_peak(po), cm.camelot_alloc_peak(pc))
    o = OA.alloc_peak(po)
    _same(OA.alloc_min(po, o.thr_num, o.thr_den * 5), cm.camelot_alloc_min(pc, o.thr_num, o.thr_den * 5))


def test_eval_and_even_split():
    lat = np.ones((3, 32, 1), np.int64) * 1000
    lat[0] = 3000
    z = np.zeros_like(lat)
    po, pc = _both(lat, z, np.zeros((3, 1)), [4], 256, 8)
    ev = OA.even_split(po, 0)
    ok, a = cm.camelot_alloc_eval(pc, 0, [1, 1, 1], ev.cu)
    assert ok
    _same(ev, a)
    ok, _ = cm.camelot_alloc_eval(pc, 0, [1, 1, 1], [128, 128, 8])
    assert not ok


def test_invalid_problems_rejected():
    lat = np.ones((1, 4, 1), np.int64)
    for kw in (dict(cu_total=30, cu_step=8), dict(cu_total=0, cu_step=8)):
        p = cm.ProblemArrays(max_instances=4, max_inst_per_stage=1, batches=[1], qos_ns=10, hbm_bytes_budget=1,
                             hbm_bw_budget=1, lat_ns=lat, bw_bps=np.zeros_like(lat), mem_bytes=np.zeros((1, 1)),
                             **kw)
        with pytest.raises(cm.CamelotError) as e:
            cm.camelot_alloc_peak(p)
        assert e.value.code == cm.EINVAL
    p = cm.ProblemArrays(cu_total=32, cu_step=8, max_instances=4, max_inst_per_stage=1, batches=[1], qos_ns=10,
                         hbm_bytes_budget=1, hbm_bw_budget=1, lat_ns=lat, bw_bps=-np.ones_like(lat),
                         mem_bytes=np.zeros((1, 1)))
    with pytest.raises(cm.CamelotError):
        cm.camelot_alloc_peak(p)


@pytest.mark.parametrize("sub", range(6))
def test_per_stage_instance_bounds_match_brute_force(sub):
    g = G.rng("tables", 77, sub)
    S = int(g.integers(2, 4))
    K = int(g.integers(2, 6))
    lat, bw, mem = G.random_problem_tables(S, K, [1, 4], seed=11, sub=sub)
    inst_max = [int(v) for v in g.integers(1, 4, S)]
    po, pc = _both(lat, bw, mem, [1, 4], K * 8, 8, nmax=3, I=3 * S, inst_max=inst_max)
    o = OA.alloc_peak(po)
    _same(o, cm.camelot_alloc_peak(pc))
    if o is not None:
        assert all(n <= m for n, m in zip(o.n, inst_max))
        lam = o.thr_num // (2 * o.thr_den) + 1
        _same(OA.alloc_min(po, lam, 1), cm.camelot_alloc_min(pc, lam, 1))


def _sa_case(sub):
    """A random problem of up to 5 stages (beyond what a test enumerates quickly for
    the larger ones), with bandwidth, memory and QoS constraints that bind."""
    g = G.rng("tables", 123, sub)
    S = int(g.integers(2, 6))
    K = int(g.integers(4, 17))
    batches = [1, 4, 16, 64][: int(g.integers(2, 5))]
    lat, bw, mem = G.random_problem_tables(S, K, batches, seed=11, sub=sub)
    lat[g.random(lat.shape) < 0.05] = 0
    nmax = int(g.integers(1, 5))
    tot = int(np.sum(np.max(lat, axis=(1, 2))))
    kw = dict(nmax=nmax, I=int(g.integers(S, S * nmax + 1)), qos=int(tot * g.uniform(0.4, 1.2)),
              bw_budget=int(np.sum(np.max(bw, axis=(1, 2))) * g.uniform(0.5, 2.0)),
              mem_budget=int(np.sum(mem) * g.uniform(0.5, 2.0)))
    return _both(lat, bw, mem, batches, 8 * K, 8, **kw)


@pytest.mark.parametrize("sub", range(10))
def test_annealing_matches_the_oracle(sub):
    """Same problem, objective, iterations and seed: the library's annealing and the
    oracle's visit the same states (one SplitMix64 stream) and return the same bits."""
    po, pc = _sa_case(sub)
    for seed in (0, 1 + sub):
        o = OA.simulated_annealing(po, 3000, seed)
        c = cm.camelot_alloc_sa(pc, cm.OBJ_PEAK, iters=3000, seed=seed)
        _same(o, c)
        if o is not None:
            lam = o.thr / 2
            o2 = OA.simulated_annealing(po, 3000, seed, load=lam)
            c2 = cm.camelot_alloc_sa(pc, cm.OBJ_MIN, lam.numerator, lam.denominator, iters=3000, seed=seed)
            _same(o2, c2)


def test_annealing_arguments():
    po, pc = _sa_case(0)
    with pytest.raises(cm.CamelotError):
        cm.camelot_alloc_sa(pc, 7)
    with pytest.raises(cm.CamelotError):
        cm.camelot_alloc_sa(pc, cm.OBJ_MIN, 1, 0)
    with pytest.raises(cm.CamelotError):
        cm.camelot_alloc_sa(pc, cm.OBJ_PEAK, iters=-1)
