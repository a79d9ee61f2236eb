"""Several instances of one stage (N_i > 1 in the allocation of Sec. 5): instance j of
a stage with N instances takes batches j, j + N, ... on its own CU share, and the
rings keep batches in sequence order, so delivery is exactly-once and in order and
each row's result is bit-identical to the one-instance pipeline's."""
import numpy as np
import pytest

from oracle import stages as O
import workload_gen as G
from tests.gpu_util import c0_stages, c1_stages, log, to_dev, torch_cuda
from tests.test_gpu_pipeline import check_common, drain_all

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return torch_cuda()


@pytest.fixture(scope="module")
def cm():
    from paper_2005_02088_amd import camelot
    return camelot


def run_c1(torch, cm, n_inst, shares, handoff, n=96, ring_depth=8):
    ws, d_ws, stages = c1_stages(torch)
    audio = G.c1_audio(n, seed=33)
    da = to_dev(torch, audio)
    arr = G.poisson_arrivals_ns(n, 400_000, seed=4)
    torch.cuda.synchronize()
    log(f"c1 replay n_inst={n_inst} shares={shares} handoff={handoff}")
    cfg = cm.pipeline_config(stages, shares, max_batch=16, ring_depth=ring_depth, handoff=handoff,
                             ingest=cm.INGEST_REPLAY, idle_timeout_ns=5_000_000_000, n_inst=n_inst)
    p = cm.camelot_pipeline_create(cfg)
    try:
        cm.camelot_pipeline_replay(p, np.arange(1, n + 1), np.ones(n), arr, np.arange(n), da.data_ptr(), n)
        res = drain_all(cm, p, n)
        stats = cm.camelot_pipeline_stats_get(p)
    finally:
        und = cm.camelot_pipeline_destroy(p)
    assert und == 0 and len(res) == n
    check_common(cm, res, stats, list(range(1, n + 1)), 3)
    assert stats.batches[0] == stats.batches[1] == stats.batches[2]
    assert stats.rows[0] == stats.rows[1] == stats.rows[2] == n
    vals = np.array([list(r.val[:10]) for r in res], dtype=np.float32)
    idx = np.array([list(r.idx[:10]) for r in res])
    return ws, audio, vals, idx


@pytest.mark.parametrize("n_inst,shares,handoff", [
    ((1, 2, 1), (32, 96, 32), 0),
    ((1, 2, 1), (32, 96, 32), 1),
    ((1, 3, 1), (32, 64, 32), 0),
    ((1, 6, 1), (32, 32, 32), 0),
])
def test_c1_mlp_instances_match_single_instance(torch, cm, n_inst, shares, handoff):
    ws, audio, vals, idx = run_c1(torch, cm, n_inst, shares, handoff, ring_depth=max(8, 2 * n_inst[1]))
    # the MLP result of a row does not depend on the batch it rides in nor on the
    # instance (or CU share) that runs it, so the one-instance pipeline agrees bit for bit
    _, _, vals1, idx1 = run_c1(torch, cm, (1, 1, 1), (32, 96, 32), 0)
    assert np.array_equal(vals.view(np.uint32), vals1.view(np.uint32))
    assert np.array_equal(idx, idx1)
    scores = O.mlp_bf16(O.log_mel(audio), ws)
    _, rval = O.topk(scores, 10)
    assert O.normwise_err(vals.astype(np.float64), rval) <= 2e-2


def test_instances_rejected_where_not_allowed(torch, cm):
    _, d_ws, stages = c1_stages(torch)           # d_ws: keeps the device weights alive
    bad = [
        cm.pipeline_config(stages, (32, 32, 32), n_inst=(2, 1, 1)),              # first stage
        cm.pipeline_config(stages, (32, 32, 32), n_inst=(1, 1, 2)),              # last stage
        cm.pipeline_config(stages, (8, 16, 8), n_inst=(1, 7, 1), ring_depth=16),  # above the maximum
        cm.pipeline_config(stages, (32, 32, 32), n_inst=(1, 3, 1), ring_depth=4),  # ring too shallow
        cm.pipeline_config(stages, (32, 112, 32), n_inst=(1, 2, 1)),             # 288 CUs in all
    ]
    for cfg in bad:
        with pytest.raises(cm.CamelotError) as e:
            cm.camelot_pipeline_create(cfg)
        assert e.value.code == cm.EINVAL


def test_c0_host_ingest_unaffected_by_instance_field(torch, cm):
    """n_inst of 0 reads as one instance (a zero-initialised config stays valid)."""
    (w1, w2), dws, stages = c0_stages(torch)
    x = G.c0_queries(8, seed=9)
    torch.cuda.synchronize()
    cfg = cm.pipeline_config(stages, (16, 16), idle_timeout_ns=5_000_000_000)
    cfg.n_inst[0] = 0
    cfg.n_inst[1] = 0
    p = cm.camelot_pipeline_create(cfg)
    try:
        for i in range(8):
            cm.camelot_pipeline_submit(p, i + 1, x[i], 1)
        res = drain_all(cm, p, 8)
    finally:
        cm.camelot_pipeline_destroy(p)
    assert [r.query_id for r in res] == list(range(1, 9))


def run_c1_full_batches(torch, cm, n_inst, shares, n=768):
    """Every request arrives at once, batches of 128 rows: the MLP worker forms the
    next batch while the current one runs; on 32-CU shares the first layer rounds
    its rows into fragment order in a pass of its own."""
    ws, d_ws, stages = c1_stages(torch)
    audio = G.c1_audio(n, seed=41)
    da = to_dev(torch, audio)
    torch.cuda.synchronize()
    log(f"c1 full batches n_inst={n_inst} shares={shares}")
    cfg = cm.pipeline_config(stages, shares, max_batch=128, batch_target=128, ring_depth=max(4, 2 * n_inst[1]),
                             ingest=cm.INGEST_REPLAY, idle_timeout_ns=5_000_000_000, n_inst=n_inst,
                             egress_capacity=4096)
    p = cm.camelot_pipeline_create(cfg)
    try:
        cm.camelot_pipeline_replay(p, np.arange(1, n + 1), np.ones(n), np.zeros(n, np.int64), np.arange(n),
                                   da.data_ptr(), n)
        res = drain_all(cm, p, n)
        stats = cm.camelot_pipeline_stats_get(p)
    finally:
        und = cm.camelot_pipeline_destroy(p)
    assert und == 0 and len(res) == n
    check_common(cm, res, stats, list(range(1, n + 1)), 3)
    vals = np.array([list(r.val[:10]) for r in res], dtype=np.float32)
    idx = np.array([list(r.idx[:10]) for r in res])
    return ws, audio, vals, idx


def test_mlp_full_batches_same_bits_on_both_first_layer_paths(torch, cm):
    # 32-CU MLP shares: the first layer rounds its rows in a pass of its own; a
    # 64-CU share: the units round them; two instances: batches alternate
    ws, audio, v32, i32 = run_c1_full_batches(torch, cm, (1, 1, 1), (32, 32, 32))
    _, _, v2x, i2x = run_c1_full_batches(torch, cm, (1, 2, 1), (32, 32, 32))
    _, _, v64, i64 = run_c1_full_batches(torch, cm, (1, 1, 1), (32, 64, 32))
    for v, i in ((v2x, i2x), (v64, i64)):
        assert np.array_equal(v.view(np.uint32), v32.view(np.uint32))
        assert np.array_equal(i, i32)
    scores = O.mlp_bf16(O.log_mel(audio[:64]), ws)
    _, rval = O.topk(scores, 10)
    assert O.normwise_err(v32[:64].astype(np.float64), rval) <= 2e-2
