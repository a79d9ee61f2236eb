"""A peer process for cross-process handoff on one GPU: it opens what another process
exported (a handoff region or a pipeline's output ring) and runs the other side.
Prints one JSON line when it is ready and one with each result; every wait is bounded.

    python -m paper_2005_02088_amd.ipc_peer consumer <handle hex> <n_slots> <cu_offset> <timeout_ms>
    python -m paper_2005_02088_amd.ipc_peer consumers      (lines of the four arguments above on stdin)
    python -m paper_2005_02088_amd.ipc_peer pipeline <handle hex> <n_rows> <cu_offset> <out .npz>
    python -m paper_2005_02088_amd.ipc_peer refuse <handle hex> <cu_offset>

`pipeline` runs a one-stage top-10 pipeline over 4096 scores per row fed by the
exported ring and saves its results; `refuse` tries to open the ring with a stage
that consumes another row size and reports the error.
"""
import json
import sys
import time

import numpy as np

# Both processes must run the same HIP runtime: an IPC handle from one runtime build
# does not open in another. In a process that imports torch first, the library runs on
# the runtime torch ships, so the peer does the same when torch is there.
try:
    import torch  # noqa: F401
except ImportError:
    pass
from paper_2005_02088_amd import camelot as cm  # noqa: E402


def say(**kw):
    print(json.dumps(kw), flush=True)


def consumer(handle, n_slots, cu_offset, timeout_ms):
    r = cm.camelot_ipc_region_open(bytes.fromhex(handle))
    try:
        say(ready=1, **cm.camelot_ipc_region_info(r))
        out = cm.camelot_ipc_handoff_run(r, cm.IPC_CONSUMER, n_slots, cu_offset, timeout_ms)
    finally:
        cm.camelot_ipc_region_destroy(r)
    say(**out)          # once the mapping is closed: the creator may free the region


def pipeline(handle, n_rows, cu_offset, out_path):
    # the downstream microservice: top-10 of the 4096 scores each row carries
    topk = cm.stage_desc(cm.STAGE_TOPK, dims=(4096,), k=10, n_layers=0)
    cfg = cm.pipeline_config([topk], [16], cu_offset=cu_offset, max_batch=16, ring_depth=4,
                             ingest=cm.INGEST_IPC, ipc_handle=bytes.fromhex(handle),
                             egress_capacity=1 << 16, idle_timeout_ns=20_000_000_000)
    p = cm.camelot_pipeline_create(cfg)
    res = []
    try:
        _, setup_ns = cm.camelot_pipeline_ipc_info(p)
        say(ready=1, setup_ns=setup_ns)
        t_end = time.monotonic() + 30
        while len(res) < n_rows and time.monotonic() < t_end:
            res += cm.camelot_pipeline_drain(p, 4096, 100_000_000)
    finally:
        und = cm.camelot_pipeline_destroy(p)
    np.savez(out_path, ids=np.array([r.query_id for r in res], np.uint64),
             rows=np.array([r.row for r in res], np.int32),
             idx=np.array([list(r.idx[:10]) for r in res], np.int32).reshape(-1, 10),
             val=np.array([list(r.val[:10]) for r in res], np.float32).reshape(-1, 10),
             t_ns=np.array([list(r.t_ns) for r in res], np.uint64).reshape(len(res), -1))
    say(done=len(res), undelivered=und)


def refuse(handle, cu_offset):
    # a stage 0 that consumes 2048-score rows cannot read a ring of 4096-score rows
    small = cm.stage_desc(cm.STAGE_TOPK, dims=(2048,), k=10, n_layers=0)
    cfg = cm.pipeline_config([small], [16], cu_offset=cu_offset, max_batch=16, ring_depth=4,
                             ingest=cm.INGEST_IPC, ipc_handle=bytes.fromhex(handle),
                             idle_timeout_ns=2_000_000_000)
    try:
        p = cm.camelot_pipeline_create(cfg)
    except cm.CamelotError as e:
        say(code=e.code, msg=str(e))
        return
    cm.camelot_pipeline_destroy(p)
    say(code=0, msg="created")


if __name__ == "__main__":
    mode = sys.argv[1]
    if mode == "consumer":
        consumer(sys.argv[2], int(sys.argv[3]), int(sys.argv[4]), int(sys.argv[5]))
    elif mode == "consumers":
        for line in sys.stdin:
            if line.strip():
                h, n, off, tmo = line.split()
                consumer(h, int(n), int(off), int(tmo))
    elif mode == "pipeline":
        pipeline(sys.argv[2], int(sys.argv[3]), int(sys.argv[4]), sys.argv[5])
    elif mode == "refuse":
        refuse(sys.argv[2], int(sys.argv[3]))
    else:
        raise SystemExit(f"unknown mode {mode}")
