"""Helpers shared by the GPU tests (device buffers via torch, library calls via the binding)."""
import functools
import sys

import numpy as np


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def torch_cuda():
    import pytest
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def to_dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def c0_stages(torch, seed=0):
    """Device weights and stage descriptors of the two-stage FP32 pipeline. The
    descriptors hold raw pointers: the caller keeps the returned device tensors
    alive for as long as it uses them."""
    import workload_gen as G
    from paper_2005_02088_amd import camelot as cm
    w1, w2 = G.c0_weights(seed)
    d_w1, d_w2 = to_dev(torch, w1), to_dev(torch, w2)
    a = cm.stage_desc(cm.STAGE_GEMM_RELU, dims=(512, 512), weights=(d_w1.data_ptr(),))
    b = cm.stage_desc(cm.STAGE_GEMM_ARGMAX, dims=(512, 10), weights=(d_w2.data_ptr(),))
    return (w1, w2), (d_w1, d_w2), (a, b)


@functools.lru_cache(maxsize=4)
def c1_weights(seed=0):
    import workload_gen as G
    return G.c1_mlp_weights(seed)


def c1_stages(torch, seed=0, k=10):
    """Device weights and stage descriptors of the speech-assistant pipeline (keep
    the returned device tensors alive while the descriptors are in use)."""
    import workload_gen as G
    from paper_2005_02088_amd import camelot as cm
    ws = c1_weights(seed)
    d_ws = [to_dev(torch, w.view(np.int16)) for w in ws]
    mel = cm.stage_desc(cm.STAGE_LOGMEL, n_layers=0)
    mlp = cm.stage_desc(cm.STAGE_MLP_BF16, dims=G.C1_MLP_DIMS, weights=[t.data_ptr() for t in d_ws])
    top = cm.stage_desc(cm.STAGE_TOPK, dims=(G.C1_MLP_DIMS[-1],), k=k, n_layers=0)
    return ws, d_ws, (mel, mlp, top)
