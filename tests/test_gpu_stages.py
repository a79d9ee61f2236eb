"""Stage kernels on the GPU vs the FP64 oracle (called through the C ABI).

Tolerances (normwise max|y - r| / max|r|): 1e-5 for FP32 stages, 2e-2 for the BF16
MLP; top-k and argmax are exact on identical inputs."""
import numpy as np
import pytest

from oracle import stages as O
import workload_gen as G
from tests.gpu_util import c0_stages, c1_stages, log, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return torch_cuda()


@pytest.fixture(scope="module")
def cm():
    from paper_2005_02088_amd import camelot
    return camelot


def test_every_stage_kernel_fits_twice_per_cu(torch, cm):
    """Workers launch one workgroup per CU of a share but need room for two (the
    dispatcher may double up on a CU); every stage kernel stays within that."""
    kinds = (cm.STAGE_GEMM_RELU, cm.STAGE_GEMM_ARGMAX, cm.STAGE_LOGMEL, cm.STAGE_MLP_BF16, cm.STAGE_TOPK,
             cm.STAGE_GATHER, cm.STAGE_CONV_POOL, cm.STAGE_GATHER_SCORE)
    for kind in kinds:
        for one_shot in (True, False):
            info = cm.camelot_stage_kernel_info(kind, one_shot)
            log(f"  kind {kind} one_shot={one_shot}: {info}")
            assert info["fits"] and info["regs"] <= 256 and info["lds_bytes"] <= 80 * 1024


def test_device_query(torch, cm):
    d = cm.camelot_device_query()
    log(f"device: {d.arch} CUs={d.n_cus} wallclock={d.wall_clock_hz} hbm={d.hbm_bytes >> 30} GiB")
    assert d.n_cus >= 8 and d.wall_clock_hz > 0


@pytest.mark.parametrize("rows", [1, 7, 32, 128])
def test_gemm_relu_parity(torch, cm, rows):
    (w1, _), dws, (sa, _) = c0_stages(torch)      # dws: keeps the device weights alive
    x = G.c0_queries(rows, seed=rows)
    dx = to_dev(torch, x)
    dy = torch.empty((rows, 512), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    log(f"gemm_relu rows={rows}")
    cm.camelot_stage_run(sa, dx.data_ptr(), dy.data_ptr(), rows, 64, 0)
    y = dy.cpu().numpy()
    err = O.normwise_err(y, O.gemm_relu(x, w1))
    log(f"  err={err:.3e}")
    assert err <= 1e-5


def test_gemm_relu_grid_and_batch_invariant(torch, cm):
    (w1, _), dws, (sa, _) = c0_stages(torch)      # dws: keeps the device weights alive
    x = G.c0_queries(32, seed=5)
    dx = to_dev(torch, x)
    outs = []
    for n_cus, rows in ((8, 32), (128, 32), (256, 32), (64, 1)):
        dy = torch.empty((rows, 512), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        cm.camelot_stage_run(sa, dx.data_ptr(), dy.data_ptr(), rows, n_cus, 0)
        outs.append(dy.cpu().numpy())
    for o in outs[1:3]:
        assert np.array_equal(o, outs[0])
    assert np.array_equal(outs[3][0], outs[0][0])


@pytest.mark.parametrize("k,n", [(100, 200), (1024, 64), (16, 17), (7, 130)])
def test_gemm_relu_ragged_shapes(torch, cm, k, n):
    """Input widths that leave a short K chunk per wave (not a multiple of 16 or of
    64) and output widths that leave a partial 64-column block."""
    g = G.rng("c0_weights", 77, k)
    w = (g.standard_normal((k, n)) / np.sqrt(k)).astype(np.float32)
    x = g.standard_normal((13, k)).astype(np.float32)
    dw, dx = to_dev(torch, w), to_dev(torch, x)
    dy = torch.empty((13, n), dtype=torch.float32, device="cuda")
    desc = cm.stage_desc(cm.STAGE_GEMM_RELU, dims=(k, n), weights=(dw.data_ptr(),))
    torch.cuda.synchronize()
    log(f"gemm_relu ragged k={k} n={n}")
    cm.camelot_stage_run(desc, dx.data_ptr(), dy.data_ptr(), 13, 16, 0)
    err = O.normwise_err(dy.cpu().numpy(), O.gemm_relu(x, w))
    log(f"  err={err:.3e}")
    assert err <= 1e-5


@pytest.mark.parametrize("rows", [1, 9, 64])
def test_gemm_argmax_parity(torch, cm, rows):
    (w1, w2), dws, (sa, sb) = c0_stages(torch)    # dws: keeps the device weights alive
    x = G.c0_queries(rows, seed=100 + rows)
    dx = to_dev(torch, x)
    dy = torch.empty((rows, 512), dtype=torch.float32, device="cuda")
    dout = torch.empty(2 * rows, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    cm.camelot_stage_run(sa, dx.data_ptr(), dy.data_ptr(), rows, 32, 0)
    cm.camelot_stage_run(sb, dy.data_ptr(), dout.data_ptr(), rows, 32, 0)
    y = dy.cpu().numpy()
    raw = dout.cpu().numpy()
    idx = raw[:rows]
    val = raw[rows:].view(np.float32)
    s, ref = O.gemm_argmax(y, w2)        # on the GPU's own stage-A output
    srt = np.sort(s, axis=1)
    gap = srt[:, -1] - srt[:, -2]
    tol = 1e-5 * np.max(np.abs(s))
    sure = gap > tol
    assert np.array_equal(idx[sure], ref[sure])
    assert O.normwise_err(val, s[np.arange(rows), ref]) <= 1e-5


def test_topk_parity_with_ties(torch, cm):
    g = G.rng("handoff", 31)
    # the candidate filter (k <= 64), direct ranking (N <= 256) and the k-round path
    # (k > 64 with N > 256, or rows of equal values: every element passes the filter)
    for rows, n, k, zero in ((1, 4096, 10, False), (13, 4096, 10, False), (64, 4096, 100, False),
                             (5, 256, 100, False), (3, 100, 100, False), (4, 37, 5, False),
                             (2, 4096, 10, True), (2, 200, 64, True), (3, 4096, 64, False)):
        s = np.round(g.standard_normal((rows, n)), 2).astype(np.float32)   # many exact ties
        if zero:
            s[:] = 0.0
        ds = to_dev(torch, s)
        dout = torch.empty(2 * rows * k, dtype=torch.int32, device="cuda")
        desc = cm.stage_desc(cm.STAGE_TOPK, dims=(n,), k=k, n_layers=0)
        torch.cuda.synchronize()
        log(f"topk rows={rows} n={n} k={k} zero={zero}")
        cm.camelot_stage_run(desc, ds.data_ptr(), dout.data_ptr(), rows, 16, 0)
        raw = dout.cpu().numpy()
        idx = raw[: rows * k].reshape(rows, k)
        val = raw[rows * k:].view(np.float32).reshape(rows, k)
        ridx, rval = O.topk(s, k)
        assert np.array_equal(idx, ridx)
        assert np.array_equal(val, rval)


@pytest.mark.parametrize("rows", [1, 3, 16])
def test_logmel_parity(torch, cm, rows):
    audio = G.c1_audio(rows, seed=rows)
    da = to_dev(torch, audio)
    dy = torch.empty((rows, 440), dtype=torch.float32, device="cuda")
    desc = cm.stage_desc(cm.STAGE_LOGMEL, n_layers=0)
    torch.cuda.synchronize()
    log(f"logmel rows={rows}")
    cm.camelot_stage_run(desc, da.data_ptr(), dy.data_ptr(), rows, 32, 0)
    y = dy.cpu().numpy()
    err = O.normwise_err(y, O.log_mel(audio))
    log(f"  err={err:.3e}")
    assert err <= 1e-5


def test_logmel_batch_and_grid_invariant(torch, cm):
    """A row's log-mel frames are bit-identical alone and at any position of any batch,
    on any share (the frames of a batch are spread over waves in pairs, so a frame
    runs in either slot of a pair)."""
    audio = G.c1_audio(37, seed=11)
    da = to_dev(torch, audio)
    desc = cm.stage_desc(cm.STAGE_LOGMEL, n_layers=0)
    full = torch.empty((37, 440), dtype=torch.float32, device="cuda")
    one = torch.empty((1, 440), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    cm.camelot_stage_run(desc, da.data_ptr(), full.data_ptr(), 37, 32, 0)
    f = full.cpu().numpy()
    for share in (8, 16, 64):
        for r in (0, 5, 36):
            cm.camelot_stage_run(desc, da[r:r + 1].data_ptr(), one.data_ptr(), 1, share, 0)
            assert np.array_equal(one.cpu().numpy()[0].view(np.uint32), f[r].view(np.uint32)), (share, r)
        part = torch.empty((20, 440), dtype=torch.float32, device="cuda")
        cm.camelot_stage_run(desc, da[9:29].data_ptr(), part.data_ptr(), 20, share, 0)
        assert np.array_equal(part.cpu().numpy().view(np.uint32), f[9:29].view(np.uint32)), share


def test_logmel_silence_and_impulse(torch, cm):
    audio = np.zeros((2, 2000), np.float32)
    audio[1, 170] = 1.0
    da = to_dev(torch, audio)
    dy = torch.empty((2, 440), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    cm.camelot_stage_run(cm.stage_desc(cm.STAGE_LOGMEL, n_layers=0), da.data_ptr(), dy.data_ptr(), 2, 8, 0)
    y = dy.cpu().numpy()
    ref = O.log_mel(audio)
    assert O.normwise_err(y, ref) <= 1e-5
    assert np.all(np.abs(y[0] - np.log(1e-10)) < 1e-5 * abs(np.log(1e-10)))


@pytest.mark.parametrize("rows", [1, 5, 16, 40, 77, 128])
def test_mlp_bf16_parity(torch, cm, rows):
    ws, d_ws, (_, mlp, _) = c1_stages(torch)
    x = O.log_mel(G.c1_audio(min(rows, 4), seed=40 + rows)).astype(np.float32)
    x = np.tile(x, (rows // len(x) + 1, 1))[:rows]
    x = x + G.rng("handoff", rows).standard_normal(x.shape).astype(np.float32)
    dx = to_dev(torch, x)
    dy = torch.empty((rows, 4096), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    log(f"mlp rows={rows}")
    ns = cm.camelot_stage_run(mlp, dx.data_ptr(), dy.data_ptr(), rows, 128, 0)
    y = dy.cpu().numpy()
    err = O.normwise_err(y, O.mlp_bf16(x, ws))
    log(f"  err={err:.3e} ns={ns:.0f}")
    assert err <= 2e-2


def test_mlp_batch_and_grid_invariant(torch, cm):
    ws, d_ws, (_, mlp, _) = c1_stages(torch)
    x = G.rng("handoff", 77).standard_normal((128, 440)).astype(np.float32)
    dx = to_dev(torch, x)
    full = torch.empty((128, 4096), dtype=torch.float32, device="cuda")
    one = torch.empty((1, 4096), dtype=torch.float32, device="cuda")
    other = torch.empty((128, 4096), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    cm.camelot_stage_run(mlp, dx.data_ptr(), full.data_ptr(), 128, 128, 0)
    cm.camelot_stage_run(mlp, dx[37:38].data_ptr(), one.data_ptr(), 1, 64, 64)
    cm.camelot_stage_run(mlp, dx.data_ptr(), other.data_ptr(), 128, 48, 200 - 48 - 8)
    f = full.cpu().numpy()
    assert np.array_equal(one.cpu().numpy()[0], f[37])
    assert np.array_equal(other.cpu().numpy(), f)
    # every unit shape (shares 8 .. 256, batches above and below 4 row blocks) gives
    # the same bits for a row
    for share in (8, 64, 128, 256):
        cm.camelot_stage_run(mlp, dx.data_ptr(), other.data_ptr(), 128, share, 0)
        assert np.array_equal(other.cpu().numpy(), f), share
    for lo, n in ((3, 40), (11, 77), (50, 49)):
        part = torch.empty((n, 4096), dtype=torch.float32, device="cuda")
        cm.camelot_stage_run(mlp, dx[lo:lo + n].data_ptr(), part.data_ptr(), n, 64, 0)
        assert np.array_equal(part.cpu().numpy(), f[lo:lo + n]), (lo, n)


@pytest.mark.parametrize("share", [8, 64, 256])
def test_mlp_bf16_narrow_layers_and_k_tails(torch, cm, share):
    """Layer widths that are odd multiples of 16 (one-strip units, K tails of 16 in
    the next layer) and an input width that is not a multiple of 32."""
    dims = (200, 144, 208, 48)
    ws = G.c1_mlp_weights(3, dims=dims)
    d_ws = [to_dev(torch, w.view(np.int16)) for w in ws]
    mlp = cm.stage_desc(cm.STAGE_MLP_BF16, dims=dims, weights=[t.data_ptr() for t in d_ws])
    x = G.rng("handoff", 91).standard_normal((100, 200)).astype(np.float32)
    dx = to_dev(torch, x)
    dy = torch.empty((100, 48), dtype=torch.float32, device="cuda")
    one = torch.empty((1, 48), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    log(f"mlp narrow share={share}")
    cm.camelot_stage_run(mlp, dx.data_ptr(), dy.data_ptr(), 100, share, 0)
    cm.camelot_stage_run(mlp, dx[93:94].data_ptr(), one.data_ptr(), 1, share, 0)
    y = dy.cpu().numpy()
    assert O.normwise_err(y, O.mlp_bf16(x, ws)) <= 2e-2
    assert np.array_equal(one.cpu().numpy()[0], y[93])


def test_stage_run_rejects_bad_shares(torch, cm):
    desc = cm.stage_desc(cm.STAGE_LOGMEL, n_layers=0)
    for n_cus, off in ((12, 0), (8, 4), (256, 8)):
        with pytest.raises(cm.CamelotError) as e:
            cm.camelot_stage_run(desc, 0, 0, 0, n_cus, off)
        assert e.value.code == cm.EINVAL
