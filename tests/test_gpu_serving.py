"""Serving: several pipelines co-located on one GPU under one HBM budget, requests of
uneven size batched continuously; a request's result is the same alone and in the mix."""
import time

import numpy as np
import pytest

from oracle import delivery as OD
from oracle import stages as O
import workload_gen as G
from tests.gpu_util import c0_stages, c1_stages, log, to_dev, torch_cuda

pytestmark = pytest.mark.gpu

TABLE_ROWS = 1 << 20


@pytest.fixture(scope="module")
def torch():
    return torch_cuda()


@pytest.fixture(scope="module")
def cm():
    from paper_2005_02088_amd import camelot
    return camelot


@pytest.fixture(scope="module")
def world(torch, cm):
    """Weights, stage descriptors and payload pools of the four pipelines."""
    w = {}
    (w1, w2), d0, s0 = c0_stages(torch)
    ws1, d1, s1 = c1_stages(torch)
    table = G.fp16_table(TABLE_ROWS, 128, seed=1)
    g = G.rng("c4", 7, 3)
    wg = (g.standard_normal((128, 512)) / np.sqrt(128)).astype(np.float32)
    dt, dwg = to_dev(torch, table.view(np.int16)), to_dev(torch, wg)
    s2 = (cm.stage_desc(cm.STAGE_GATHER, dims=(32, 128), weights=(dt.data_ptr(),), k=TABLE_ROWS),
          cm.stage_desc(cm.STAGE_GEMM_RELU, dims=(128, 512), weights=(dwg.data_ptr(),)),
          cm.stage_desc(cm.STAGE_TOPK, dims=(512,), k=10, n_layers=0))
    ws3 = G.c1_mlp_weights(3, dims=(440, 1024, 1024, 1024))
    d3 = [to_dev(torch, x.view(np.int16)) for x in ws3]
    s3 = (cm.stage_desc(cm.STAGE_LOGMEL, n_layers=0),
          cm.stage_desc(cm.STAGE_MLP_BF16, dims=(440, 1024, 1024, 1024), weights=[t.data_ptr() for t in d3]),
          cm.stage_desc(cm.STAGE_TOPK, dims=(1024,), k=10, n_layers=0))
    n_rows = 1024
    pools = [G.c0_queries_fast(n_rows, seed=4), G.c1_audio_fast(n_rows, seed=4),
             G.zipf_ids(n_rows, 32, TABLE_ROWS, seed=4), G.c1_audio_fast(n_rows, seed=5)]
    w.update(stages=[s0, s1, s2, s3], cus=[(16, 16), (16, 64, 16), (16, 16, 16), (16, 32, 16)],
             offsets=[0, 32, 128, 176], pools=pools, dpools=[to_dev(torch, p) for p in pools],
             keep=[d0, d1, dt, dwg, d3], w0=(w1, w2), ws1=ws1, table=table, wg=wg, ws3=ws3)
    torch.cuda.synchronize()
    return w


def _cfg(cm, world, i, **kw):
    return cm.pipeline_config(world["stages"][i], world["cus"][i], cu_offset=world["offsets"][i], max_batch=128,
                              batch_target=1, ring_depth=4, ingest=cm.INGEST_REPLAY, max_rows_per_request=128,
                              idle_timeout_ns=5_000_000_000, **kw)


def _drain(cm, p, n, timeout_s=20.0):
    out = []
    t_end = time.monotonic() + timeout_s
    while len(out) < n and time.monotonic() < t_end:
        out += cm.camelot_pipeline_drain(p, 4096, 100_000_000)
    return out


def test_admission_by_hbm_footprint(torch, cm, world):
    big = cm.camelot_server_create(1 << 40)
    used = []
    try:
        for i in range(4):
            assert cm.camelot_server_admit(big, _cfg(cm, world, i)) is not None
            used.append(cm.camelot_server_used_bytes(big))
    finally:
        cm.camelot_server_destroy(big)
    sizes = np.diff([0] + used)
    log(f"  footprints (MB): {np.round(sizes / 1e6, 1)}")
    # the table (256 MB) dominates pipeline 2; the speech MLP's 35 MB of weights count
    assert sizes[2] > 256e6 and sizes[1] > 35e6
    # a budget that holds pipelines 0, 1, 3 but not also 2 (one byte short)
    budget = int(sizes[0] + sizes[1] + sizes[2] + sizes[3] - 1)
    s = cm.camelot_server_create(budget)
    try:
        p0 = cm.camelot_server_admit(s, _cfg(cm, world, 0))
        p1 = cm.camelot_server_admit(s, _cfg(cm, world, 1))
        p3 = cm.camelot_server_admit(s, _cfg(cm, world, 3))
        assert None not in (p0, p1, p3)
        assert cm.camelot_server_admit(s, _cfg(cm, world, 2)) is None          # does not fit
        cm.camelot_server_release(s, p1)
        assert cm.camelot_server_admit(s, _cfg(cm, world, 2)) is not None      # fits once freed
        # a second instance sharing pipeline 0's weights only adds its own rings; it
        # takes CUs 32..63, left free by pipeline 1 (pipeline 2 now holds 128..175)
        before = cm.camelot_server_used_bytes(s)
        cfg = _cfg(cm, world, 0)
        cfg.cu_offset = 32
        assert cm.camelot_server_admit(s, cfg) is not None
        assert cm.camelot_server_used_bytes(s) - before < 10e6
        with pytest.raises(cm.CamelotError):                                   # overlapping CUs
            cm.camelot_server_admit(s, _cfg(cm, world, 0))
    finally:
        cm.camelot_server_destroy(s)


def _reference(world, i, rows):
    pool = world["pools"][i]
    if i == 0:
        s, ref = O.gemm_argmax(O.gemm_relu(pool[rows], world["w0"][0]), world["w0"][1])
        return ref[:, None], s[np.arange(len(rows)), ref][:, None]
    if i == 1:
        return O.topk(O.mlp_bf16(O.log_mel(pool[rows]), world["ws1"]), 10)
    if i == 2:
        return O.topk(O.gemm_relu(O.gather_mean(pool[rows], world["table"]), world["wg"]), 10)
    return O.topk(O.mlp_bf16(O.log_mel(pool[rows]), world["ws3"]), 10)


def _plan(world, i, nreq, start_ns, rate_qps):
    """Request plan of pipeline i: uneven sizes, Poisson arrivals from start_ns."""
    rows = G.request_rows(nreq, seed=10 + i)
    arr = start_ns + G.poisson_arrivals_ns(nreq, rate_qps, seed=i)
    prow = np.concatenate([[0], np.cumsum(rows)[:-1]]) % (len(world["pools"][i]) - 128)
    ids = np.arange(1, nreq + 1)
    return ids, rows, arr, prow


def _run_rows(cm, p, world, i, plan):
    ids, rows, arr, prow = plan
    cm.camelot_pipeline_replay(p, ids, rows, arr, prow, world["dpools"][i].data_ptr(), len(world["pools"][i]))


def _collect(cm, p, plan, timeout_s=60.0):
    ids, rows, _, _ = plan
    res = _drain(cm, p, int(rows.sum()), timeout_s=timeout_s)
    assert len(res) == int(rows.sum())
    want_ids = [int(q) for q in ids]
    assert OD.check_delivery(want_ids, list(dict.fromkeys(r.query_id for r in res))) == []
    return res


def test_alone_vs_mix_bit_identical(torch, cm, world):
    # Every pipeline serves the same request plan twice: alone on the GPU, then with
    # the other three admitted and served at the same time. All four mixed replays are
    # started before any request arrives (arrivals begin 30 ms after each pipeline's
    # start; the four starts are well under a millisecond apart), and the arrival rate
    # exceeds what each pipeline serves, so every pipeline works through a backlog
    # while the others do. Batches form differently in the two runs; the kernels are
    # batch-invariant, so every row's result must carry the same bits.
    nreq, start_ns, rate = 400, 30_000_000, 200_000
    plans = [_plan(world, i, nreq, start_ns, rate) for i in range(4)]
    alone = {}
    for i in range(4):
        p = cm.camelot_pipeline_create(_cfg(cm, world, i))
        try:
            _run_rows(cm, p, world, i, plans[i])
            res = _collect(cm, p, plans[i])
        finally:
            cm.camelot_pipeline_destroy(p)
        alone[i] = {(r.query_id, r.row): (list(r.idx[:r.n_out]), list(r.val[:r.n_out])) for r in res}
    server = cm.camelot_server_create(1 << 40)
    mixed, batches = {}, {}
    try:
        handles = [cm.camelot_server_admit(server, _cfg(cm, world, i)) for i in range(4)]
        for i, p in enumerate(handles):
            _run_rows(cm, p, world, i, plans[i])
        for i, p in enumerate(handles):
            res = _collect(cm, p, plans[i])
            mixed[i] = {(r.query_id, r.row): (list(r.idx[:r.n_out]), list(r.val[:r.n_out])) for r in res}
            # each batch's stage intervals on the common device clock, keyed by the
            # batch's first-stage start
            S = len(world["stages"][i])
            epoch = cm.camelot_pipeline_epoch_ns(p)
            b = {}
            for r in res:
                b.setdefault(r.t_ns[1], (r.query_id, [(epoch + r.t_ns[1 + 2 * s], epoch + r.t_ns[2 + 2 * s])
                                                      for s in range(S)]))
            batches[i] = list(b.values())
            # a sample request of the mix against the oracle
            ids, rows, _, prow = plans[i]
            q = 5
            got = sorted((r for r in res if r.query_id == int(ids[q])), key=lambda r: r.row)
            ridx, rval = _reference(world, i, np.arange(prow[q], prow[q] + rows[q]))
            gval = np.array([list(r.val[:r.n_out]) for r in got], np.float64)
            assert O.normwise_err(gval, rval) <= (2e-2 if i in (1, 3) else 1e-5)
    finally:
        cm.camelot_server_destroy(server)
    # the pipelines ran at the same time: for every pipeline, count the batches whose
    # stage intervals overlap some stage interval of another pipeline
    spans = {i: np.array([iv for _, ivs in batches[i] for iv in ivs], np.int64) for i in range(4)}
    for i in range(4):
        others = np.concatenate([spans[j] for j in range(4) if j != i])
        over = [q for q, ivs in batches[i]
                if any(np.any((others[:, 0] < e) & (others[:, 1] > s)) for s, e in ivs)]
        log(f"  pipeline {i}: {len(over)} of its {len(batches[i])} batches overlap other pipelines' stage work")
        assert len(over) >= max(1, len(batches[i]) // 10), f"pipeline {i} ran mostly alone"
    for i in range(4):
        assert mixed[i].keys() == alone[i].keys()
        diff = [k for k in alone[i] if mixed[i][k] != alone[i][k]]
        assert not diff, f"pipeline {i}: {len(diff)} rows differ alone vs in the mix, first {diff[:3]}"
    log(f"  all {sum(len(a) for a in alone.values())} rows bit-identical alone and in the 4-pipeline mix")
