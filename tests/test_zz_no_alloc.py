"""The allocation-free stage run (camelot_stage_run_noalloc) against camelot_stage_run:
the same kernels on the same inputs give the same bits, call after call, with the
static scratch array reused (the second call of each pair has a smaller input)."""
import numpy as np
import pytest

from oracle import stages as O
import workload_gen as G
from tests.gpu_util import c1_stages, log, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return torch_cuda()


@pytest.fixture(scope="module")
def cm():
    from paper_2005_02088_amd import camelot
    return camelot


def _both(torch, cm, desc, x, rows, out_shape, out_dtype, n_cus):
    """Runs the stage through both entry points on the same device input."""
    dx = to_dev(torch, x)
    ref = torch.full(out_shape, -7, dtype=out_dtype, device="cuda")
    got = torch.full(out_shape, -7, dtype=out_dtype, device="cuda")
    torch.cuda.synchronize()
    cm.camelot_stage_run(desc, dx.data_ptr(), ref.data_ptr(), rows, n_cus, 0)
    s = torch.cuda.Stream()
    log(f"  noalloc kind={desc.kind} rows={rows} n_cus={n_cus}")
    cm.camelot_stage_run_noalloc(desc, dx.data_ptr(), got.data_ptr(), rows, n_cus, 1, s.cuda_stream)
    s.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy()


def test_noalloc_mlp_matches_stage_run(torch, cm):
    ws, dws, (_, mlp, _) = c1_stages(torch)          # dws keeps the device weights alive
    for rows in (128, 5):
        x = G.c1_audio_fast(rows, seed=rows)
        feats = O.log_mel(x).astype(np.float32)
        ref, got = _both(torch, cm, mlp, feats, rows, (rows, 4096), torch.float32, 32)
        assert np.array_equal(ref.view(np.uint32), got.view(np.uint32))
        err = O.normwise_err(got, O.mlp_bf16(feats, ws))
        log(f"  mlp rows={rows}: bit-identical, err vs oracle {err:.2e}")
        assert err <= 2e-2


def test_noalloc_conv_matches_stage_run(torch, cm):
    wc = G.c4_conv_weights(0)
    dw = to_dev(torch, wc.view(np.int16))
    for rows, (h, w) in ((3, (G.C4_H, G.C4_W)), (2, (9, 15))):
        x = G.c4_feature_maps(rows, seed=rows, h=h, w=w)
        desc = cm.stage_desc(cm.STAGE_CONV_POOL, dims=(h, w, 64, 64), weights=(dw.data_ptr(),), n_layers=0)
        ref, got = _both(torch, cm, desc, x.view(np.int16), rows, (rows, 64), torch.float32, 64)
        assert np.array_equal(ref.view(np.uint32), got.view(np.uint32))
        err = O.normwise_err(got, O.conv3x3_relu_pool(x, wc))
        log(f"  conv {h}x{w} rows={rows}: bit-identical, err vs oracle {err:.2e}")
        assert err <= 1e-5


def test_noalloc_logmel_and_topk_match_stage_run(torch, cm):
    mel = cm.stage_desc(cm.STAGE_LOGMEL, n_layers=0)
    top = cm.stage_desc(cm.STAGE_TOPK, dims=(4096,), k=10, n_layers=0)
    for rows in (16, 3):
        x = G.c1_audio_fast(rows, seed=50 + rows)
        ref, got = _both(torch, cm, mel, x, rows, (rows, 440), torch.float32, 16)
        assert np.array_equal(ref.view(np.uint32), got.view(np.uint32))
        assert O.normwise_err(got, O.log_mel(x)) <= 1e-5
        s = G.rng("c4", 900 + rows).standard_normal((rows, 4096)).astype(np.float32)
        ref, got = _both(torch, cm, top, s, rows, (2 * rows * 10,), torch.int32, 8)
        assert np.array_equal(ref, got)
        ridx, _ = O.topk(s.astype(np.float64), 10)
        assert np.array_equal(got[:rows * 10].reshape(rows, 10), ridx)
        log(f"  logmel and top-10 rows={rows}: bit-identical")
