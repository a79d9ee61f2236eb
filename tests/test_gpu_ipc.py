"""Microservices in separate processes on one GPU (Section VI-B): batches go from one
process's stage to another process's stage through device memory the two share
(hipIpcGetMemHandle / hipIpcOpenMemHandle), with the same slot protocol as between
the stages of one pipeline. The second process is the library's peer
(paper_2005_02088_amd/ipc_peer.py); every wait on both sides is bounded."""
import json
import os
import select
import subprocess
import sys
import time

import numpy as np
import pytest

from oracle import delivery as OD
from oracle import stages as O
import workload_gen as G
from tests.gpu_util import c1_stages, log, to_dev, torch_cuda

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def torch():
    return torch_cuda()


@pytest.fixture(scope="module")
def cm():
    from paper_2005_02088_amd import camelot
    return camelot


def read_json_line(proc, timeout_s):
    """The child's next JSON line, waiting at most timeout_s."""
    t_end = time.monotonic() + timeout_s
    while time.monotonic() < t_end:
        r, _, _ = select.select([proc.stdout], [], [], 0.2)
        if r:
            line = proc.stdout.readline()
            if not line:
                break
            line = line.strip()
            if line.startswith("{"):
                return json.loads(line)
        elif proc.poll() is not None:
            break
    proc.kill()
    err = proc.stderr.read() if proc.stderr else ""
    raise AssertionError(f"child gave no result within {timeout_s} s; stderr: {err[-2000:]}")


def spawn(*args):
    return subprocess.Popen([sys.executable, "-u", "-m", "paper_2005_02088_amd.ipc_peer", *map(str, args)],
                            stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, cwd=ROOT)


@pytest.mark.parametrize("slot_bytes,depth,n_slots", [(64, 4, 2000), (65536, 4, 256), (1 << 22, 2, 16)])
def test_handoff_between_processes(torch, cm, slot_bytes, depth, n_slots):
    """The producer writes every slot in this process, the consumer reads it in the
    other: the consumer's checksum over all words is the pattern's."""
    r, handle = cm.camelot_ipc_region_create(slot_bytes, depth, 64)
    log(f"ipc handoff {slot_bytes} B x {n_slots} slots, depth {depth}: {cm.camelot_ipc_region_info(r)}")
    child = spawn("consumer", handle.hex(), n_slots, 128, 20000)
    try:
        ready = read_json_line(child, 60)
        assert ready["ready"] == 1
        prod = cm.camelot_ipc_handoff_run(r, cm.IPC_PRODUCER, n_slots, 0, 20000)
        res = read_json_line(child, 60)
        assert child.wait(timeout=30) == 0
    finally:
        if child.poll() is None:
            child.kill()
        cm.camelot_ipc_region_destroy(r)
    s, x = cm.camelot_handoff_expected(slot_bytes, n_slots)
    assert (res["sum"], res["xor"]) == (s, x)
    assert res["seconds"] > 0 and prod["seconds"] >= 0
    log(f"  open {ready['setup_ns'] / 1e3:.0f} us, {res['seconds'] * 1e6 / n_slots:.2f} us per slot, "
        f"{res['gbs']:.1f} GB/s")


def test_pipeline_split_across_processes(torch, cm):
    """log-mel -> MLP in this process, top-10 in the other, joined by an exported ring:
    every row delivered once, in submit order, with the values of the one-process
    pipeline's oracle, and stage times that follow each other across the boundary."""
    n = 600
    ws, d_ws, (mel, mlp, top) = c1_stages(torch)
    audio = G.c1_audio(n, seed=31)
    da = to_dev(torch, audio)
    arr = G.poisson_arrivals_ns(n, 100_000, seed=31)
    torch.cuda.synchronize()
    cfg = cm.pipeline_config([mel, mlp], (32, 128), max_batch=16, ring_depth=4, ingest=cm.INGEST_REPLAY,
                             idle_timeout_ns=20_000_000_000, out_ipc=True)
    p = cm.camelot_pipeline_create(cfg)
    out = os.path.join(os.environ.get("TMPDIR", "/tmp"), f"ipc_split_{os.getpid()}.npz")
    child = None
    try:
        handle, export_ns = cm.camelot_pipeline_ipc_info(p)
        with pytest.raises(cm.CamelotError) as e:       # results come out of the importer
            cm.camelot_pipeline_drain(p, 1, 0)
        assert e.value.code == cm.EINVAL
        child = spawn("pipeline", handle.hex(), n, 160, out)
        ready = read_json_line(child, 60)
        log(f"ipc split: export {export_ns / 1e3:.0f} us, open {ready['setup_ns'] / 1e3:.0f} us")
        cm.camelot_pipeline_replay(p, np.arange(1, n + 1), np.ones(n), arr, np.arange(n), da.data_ptr(), n)
        done = read_json_line(child, 90)
        assert child.wait(timeout=30) == 0
        assert done["done"] == n and done["undelivered"] == 0
    finally:
        if child is not None and child.poll() is None:
            child.kill()
        cm.camelot_pipeline_destroy(p)
    got = np.load(out)
    os.remove(out)
    ids = [int(v) for v in got["ids"]]
    assert OD.check_delivery(list(range(1, n + 1)), ids) == []
    assert np.all(got["rows"] == 0)
    # stage times: arrival, (start, end) of log-mel, MLP (this process) and top-10 (the
    # other), done; absolute device-clock ns, each no earlier than the one before
    t = got["t_ns"].astype(np.int64)
    seq = t[:, :8]
    assert np.all(np.diff(seq, axis=1) >= 0), seq[np.argmin(np.diff(seq, axis=1).min(axis=1))]
    # values: the oracle of the whole chain on a sample of rows
    m = 48
    scores = O.mlp_bf16(O.log_mel(audio[:m]), ws)
    _, rval = O.topk(scores, 10)
    assert O.normwise_err(got["val"][:m].astype(np.float64), rval) <= 2e-2
    tol = 2e-2 * np.max(np.abs(scores))
    for q in range(m):
        assert np.all(scores[q, got["idx"][q]] >= rval[q, -1] - tol)


def test_importer_refuses_a_ring_of_another_geometry(torch, cm):
    """A stage 0 that consumes another row size than the exporter produces is refused
    at create, before any worker runs (the ring's header carries its geometry)."""
    ws, d_ws, (mel, mlp, top) = c1_stages(torch)
    cfg = cm.pipeline_config([mel, mlp], (32, 64), max_batch=16, ring_depth=4, ingest=cm.INGEST_REPLAY,
                             idle_timeout_ns=2_000_000_000, out_ipc=True)
    p = cm.camelot_pipeline_create(cfg)
    child = None
    try:
        handle, _ = cm.camelot_pipeline_ipc_info(p)
        child = spawn("refuse", handle.hex(), 128)
        res = read_json_line(child, 60)
        assert child.wait(timeout=30) == 0
    finally:
        if child is not None and child.poll() is None:
            child.kill()
        cm.camelot_pipeline_destroy(p)
    assert res["code"] == cm.EINVAL and "row" in res["msg"], res
