"""The artifact suite's PCIe-, compute- and memory-intensive stages on the GPU vs the
oracle, bit for bit (their arithmetic is integer XOR, exact conversions and FP32
products and sums rounded one at a time), alone and as the pipeline p -> c -> m ->
top-10 with device-global and host-staged handoff."""
import time

import numpy as np
import pytest

from oracle import delivery as OD
from oracle import stages as O
import workload_gen as G
from tests.gpu_util import log, to_dev, torch_cuda

pytestmark = pytest.mark.gpu

D = G.ARTIFACT_D
P_TABLE_WORDS = 1 << 22          # 16 MiB of pinned host memory
M_TABLE_WORDS = 1 << 24          # 64 MiB of device memory


@pytest.fixture(scope="module")
def torch():
    return torch_cuda()


@pytest.fixture(scope="module")
def cm():
    from paper_2005_02088_amd import camelot
    return camelot


@pytest.fixture(scope="module")
def tables(torch):
    hp = G.artifact_words(P_TABLE_WORDS, seed=1)
    hm = G.artifact_words(M_TABLE_WORDS, seed=2)
    pin = torch.empty(P_TABLE_WORDS, dtype=torch.int32, pin_memory=True)
    pin.numpy()[:] = hp.view(np.int32)
    dm = to_dev(torch, hm.view(np.int32))
    torch.cuda.synchronize()
    return dict(hp=hp, hm=hm, pin=pin, dm=dm)


def _descs(cm, tables, pw, ci, mw):
    p = cm.stage_desc(cm.STAGE_ARTIFACT_P, dims=(D, pw), weights=(tables["pin"].data_ptr(),), k=P_TABLE_WORDS,
                      n_layers=0)
    c = cm.stage_desc(cm.STAGE_ARTIFACT_C, dims=(D, ci), n_layers=0)
    m = cm.stage_desc(cm.STAGE_ARTIFACT_M, dims=(D, mw), weights=(tables["dm"].data_ptr(),), k=M_TABLE_WORDS,
                      n_layers=0)
    return p, c, m


@pytest.mark.parametrize("rows,share", [(1, 8), (7, 64), (128, 32)])
def test_artifact_stages_match_the_oracle(torch, cm, tables, rows, share):
    p, c, m = _descs(cm, tables, 4096, 64, 16384)
    x = G.artifact_words(rows * D, seed=rows).reshape(rows, D)
    dx = to_dev(torch, x.view(np.int32))
    out = torch.empty((rows, D), dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    log(f"artifact stages rows={rows} share={share}")
    refs = {"p": O.artifact_fold(x, tables["hp"], 4096, False),
            "c": O.artifact_compute(x, 64),
            "m": O.artifact_fold(x, tables["hm"], 16384, True).view(np.uint32)}
    for name, desc in (("p", p), ("c", c), ("m", m)):
        cm.camelot_stage_run(desc, dx.data_ptr(), out.data_ptr(), rows, share, 0)
        got = out.cpu().numpy().view(np.uint32)
        assert np.array_equal(got, refs[name]), f"{name}: {np.count_nonzero(got != refs[name])} words differ"


def test_artifact_intensity_scales_the_work(torch, cm, tables):
    """More intense variants take longer on the same share (the knob works)."""
    x = G.artifact_words(128 * D, seed=3).reshape(128, D)
    dx = to_dev(torch, x.view(np.int32))
    out = torch.empty((128, D), dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    times = {}
    for name, args in (("c", [(D, 64), (D, 1024)]), ("m", [(D, 4096), (D, 65536)]), ("p", [(D, 1024), (D, 16384)])):
        t = []
        for dims in args:
            kind = {"p": cm.STAGE_ARTIFACT_P, "c": cm.STAGE_ARTIFACT_C, "m": cm.STAGE_ARTIFACT_M}[name]
            w = {"p": (tables["pin"].data_ptr(),), "c": (), "m": (tables["dm"].data_ptr(),)}[name]
            k = {"p": P_TABLE_WORDS, "c": 0, "m": M_TABLE_WORDS}[name]
            d = cm.stage_desc(kind, dims=dims, weights=w, k=k, n_layers=0)
            t.append(cm.camelot_stage_run(d, dx.data_ptr(), out.data_ptr(), 128, 32, 0, 4, device=True))
        times[name] = t
        assert t[1] > 2 * t[0], (name, t)
    log(f"  us per batch of 128 on 32 CUs: {({k: [round(v / 1e3, 1) for v in t] for k, t in times.items()})}")


@pytest.mark.parametrize("handoff", ["device", "host"])
def test_artifact_pipeline(torch, cm, tables, handoff):
    p, c, m = _descs(cm, tables, 4096, 256, 16384)
    top = cm.stage_desc(cm.STAGE_TOPK, dims=(D,), k=10, n_layers=0)
    n = 48
    x = G.artifact_words(n * D, seed=9).reshape(n, D)
    dx = to_dev(torch, x.view(np.int32))
    torch.cuda.synchronize()
    mode = cm.HANDOFF_DEVICE if handoff == "device" else cm.HANDOFF_HOST
    cfg = cm.pipeline_config((p, c, m, top), (16, 32, 32, 16), max_batch=16, ring_depth=4, handoff=mode,
                             ingest=cm.INGEST_REPLAY, idle_timeout_ns=5_000_000_000)
    pl = cm.camelot_pipeline_create(cfg)
    res = []
    try:
        cm.camelot_pipeline_replay(pl, np.arange(1, n + 1), np.ones(n), G.poisson_arrivals_ns(n, 100_000, seed=9),
                                   np.arange(n), dx.data_ptr(), n)
        t_end = time.monotonic() + 20
        while len(res) < n and time.monotonic() < t_end:
            res += cm.camelot_pipeline_drain(pl, 64, 100_000_000)
    finally:
        cm.camelot_pipeline_destroy(pl)
    assert OD.check_delivery(list(range(1, n + 1)), [r.query_id for r in res]) == []
    s = O.artifact_fold(O.artifact_compute(O.artifact_fold(x, tables["hp"], 4096, False), 256),
                        tables["hm"], 16384, True)
    ridx, rval = O.topk(s.astype(np.float64), 10)
    gidx = np.array([list(r.idx[:10]) for r in res])
    gval = np.array([list(r.val[:10]) for r in res], np.float64)
    assert np.array_equal(gidx, ridx) and np.array_equal(gval, rval)
    log(f"  p -> c -> m -> top-10 ({handoff} handoff): {n} queries bit-identical to the oracle")


def test_artifact_pipeline_many_instances_delivers_every_record(torch, cm, tables):
    """Regression for stale batch descriptors: five memory-stage instances side by side
    (the allocation under which a compute workgroup once wrote a batch's egress records
    from a descriptor two batches old, leaving records unwritten), 200,000 single-row
    queries offered faster than the pipeline serves them. Every record arrives whole,
    once, in submit order, and the last stage's id checksums cover every query."""
    p, c, m = _descs(cm, tables, 1024, 256, 65536)
    top = cm.stage_desc(cm.STAGE_TOPK, dims=(D,), k=10, n_layers=0)
    pool_n = 2048
    x = G.artifact_words(pool_n * D, seed=21).reshape(pool_n, D)
    dx = to_dev(torch, x.view(np.int32))
    torch.cuda.synchronize()
    n = 200_000
    cfg = cm.pipeline_config((p, c, m, top), (8, 24, 32, 8), max_batch=128, batch_target=128,
                             batch_timeout_ns=2_000_000, ring_depth=10, ingest=cm.INGEST_REPLAY,
                             egress_capacity=1 << 20, idle_timeout_ns=5_000_000_000, n_inst=(1, 1, 5, 1))
    log(f"artifact pipeline 8 / 24 / 5 x 32 / 8 CUs, {n} queries")
    pl = cm.camelot_pipeline_create(cfg)
    ids = np.empty(n, np.uint64)
    ci, cl = np.empty(1 << 16, np.uint64), np.empty(1 << 16, np.int64)
    done = 0
    try:
        cm.camelot_pipeline_replay(pl, np.arange(1, n + 1), np.ones(n), G.poisson_arrivals_ns(n, 4_000_000, seed=21),
                                   np.arange(n) % pool_n, dx.data_ptr(), pool_n)
        t_end = time.monotonic() + 30
        while done < n and time.monotonic() < t_end:
            k = cm.camelot_pipeline_drain_latency(pl, ci, cl, 100_000_000)
            ids[done:done + k] = ci[:k]
            done += k
        stats = cm.camelot_pipeline_stats_get(pl)
    finally:
        cm.camelot_pipeline_destroy(pl)
    assert done == n
    assert np.array_equal(ids, np.arange(1, n + 1, dtype=np.uint64))
    s_, x_ = OD.checksums(list(range(1, n + 1)))
    assert stats.id_sum[3] == s_ and stats.id_xor[3] == x_
    log(f"  {n} records whole and in order, batches per stage {list(stats.batches[:4])}")
