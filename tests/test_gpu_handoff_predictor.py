"""Device-global handoff benchmark (data integrity) and the predictor's GPU kernels
vs the FP64 oracle."""
import numpy as np
import pytest

from oracle import predictor as OP
from oracle import stages as O
import workload_gen as G
from tests.gpu_util import log, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return torch_cuda()


@pytest.fixture(scope="module")
def cm():
    from paper_2005_02088_amd import camelot
    return camelot


@pytest.mark.parametrize("slot,depth,n,cp,cc", [(1 << 20, 4, 64, 64, 64), (4096, 2, 33, 8, 16),
                                                (48, 3, 10, 8, 8), ((64 << 20), 16, 48, 128, 128)])
def test_handoff_device_checksum(torch, cm, slot, depth, n, cp, cc):
    log(f"handoff slot={slot} depth={depth} n={n}")
    r = cm.camelot_handoff_bench(cm.HANDOFF_DEVICE, slot, depth, n, cp, cc)
    s, x = cm.camelot_handoff_expected(slot, n)
    log(f"  {r['gbs']:.1f} GB/s in {r['seconds'] * 1e3:.2f} ms")
    assert (r["sum"], r["xor"]) == (s, x)


def test_handoff_host_staged_runs(torch, cm):
    r = cm.camelot_handoff_bench(cm.HANDOFF_HOST, 1 << 20, 2, 8, 8, 8)
    log(f"host-staged {r['gbs']:.2f} GB/s")
    assert r["gbs"] > 0


def _flat(params):
    return np.concatenate([np.asarray(p, np.float32).reshape(-1) for p in params])


def _split(flat):
    shapes = [(16, 64), (64,), (64, 64), (64,), (64, 1), (1,)]
    out, o = [], 0
    for s in shapes:
        n = int(np.prod(s))
        out.append(flat[o:o + n].reshape(s))
        o += n
    return out


@pytest.mark.parametrize("m", [1, 64, 256, 300])
def test_predictor_grad_parity(torch, cm, m):
    params = G.predictor_init(seed=1)
    params = [p + 0.05 * (i % 2) for i, p in enumerate(params)]
    x, y = G.predictor_batch(m, seed=2)
    dp, dx, dy = to_dev(torch, _flat(params)), to_dev(torch, x), to_dev(torch, y)
    dg = torch.empty(cm.PRED_NPARAMS, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    loss = cm.camelot_predictor_grad(dp.data_ptr(), dx.data_ptr(), dy.data_ptr(), m, dg.data_ptr())
    g = _split(dg.cpu().numpy())
    ref = OP.grad(params, x, y)
    for a, b in zip(g, ref):
        assert O.normwise_err(a, b) <= 1e-5
    assert abs(loss - OP.loss(params, x, y)) <= 1e-5 * OP.loss(params, x, y)
    yh = torch.empty(m, dtype=torch.float32, device="cuda")
    cm.camelot_predictor_forward(dp.data_ptr(), dx.data_ptr(), m, yh.data_ptr())
    assert O.normwise_err(yh.cpu().numpy(), OP.forward(params, x)[0]) <= 1e-5


def test_predictor_adam_parity_and_training(torch, cm):
    params = G.predictor_init(seed=3)
    x, y = G.predictor_batch(256, seed=3)
    dp, dx, dy = to_dev(torch, _flat(params)), to_dev(torch, x), to_dev(torch, y)
    z = np.zeros(cm.PRED_NPARAMS, np.float32)
    dm1, dm2 = to_dev(torch, z), to_dev(torch, z.copy())
    dg = torch.empty(cm.PRED_NPARAMS, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    # steps t = 1..3 one at a time: the GPU gradient at the GPU's parameters against
    # the oracle's, then the oracle's Adam step on the GPU's state and gradient
    # against the GPU's (parameters and both moments)
    for t in (1, 2, 3):
        p_now = _split(dp.cpu().numpy().astype(np.float64))
        m_now = _split(dm1.cpu().numpy().astype(np.float64))
        v_now = _split(dm2.cpu().numpy().astype(np.float64))
        cm.camelot_predictor_grad(dp.data_ptr(), dx.data_ptr(), dy.data_ptr(), 256, dg.data_ptr())
        g = dg.cpu().numpy()
        assert O.normwise_err(g, _flat(OP.grad(p_now, x, y))) <= 1e-5
        cm.camelot_predictor_adam(dp.data_ptr(), dg.data_ptr(), dm1.data_ptr(), dm2.data_ptr(), t, 1e-3)
        ref_p, ref_m, ref_v = OP.adam_step(p_now, _split(g.astype(np.float64)), m_now, v_now, t, lr=1e-3)
        log(f"  adam t={t}: params err {O.normwise_err(dp.cpu().numpy(), _flat(ref_p)):.2e}")
        assert O.normwise_err(dp.cpu().numpy(), _flat(ref_p)) <= 1e-5
        assert O.normwise_err(dm1.cpu().numpy(), _flat(ref_m)) <= 1e-5
        assert O.normwise_err(dm2.cpu().numpy(), _flat(ref_v)) <= 1e-5
    # a few epochs of training on a fixed set lower the loss
    t, losses = cm.camelot_predictor_train(dp.data_ptr(), dm1.data_ptr(), dm2.data_ptr(), 3, dx.data_ptr(),
                                           dy.data_ptr(), 256, 64, 100, lr=1e-2)
    log(f"  predictor loss {losses[0]:.3f} -> {losses[-1]:.4f}")
    assert t == 3 + 400
    assert losses[-1] < 0.2 * losses[0]


def test_predictor_train_loop_matches_oracle(torch, cm):
    """camelot_predictor_train over 3 epochs of shuffled minibatches (12 Adam steps,
    the last minibatch of each epoch ragged) against the oracle's own FP64 loop
    (its gradients, its Adam) from the same start: parameters and both moments."""
    n, batch, epochs, lr = 232, 64, 3, 1e-3
    params = G.predictor_init(seed=5)
    x, y = G.predictor_batch(n, seed=5)
    perm = np.stack([G.rng("predictor", 5, 2000 + e).permutation(n) for e in range(epochs)]).astype(np.int32)
    dp, dx, dy = to_dev(torch, _flat(params)), to_dev(torch, x), to_dev(torch, y)
    z = np.zeros(cm.PRED_NPARAMS, np.float32)
    dm1, dm2, dperm = to_dev(torch, z), to_dev(torch, z.copy()), to_dev(torch, perm)
    torch.cuda.synchronize()
    t, losses = cm.camelot_predictor_train(dp.data_ptr(), dm1.data_ptr(), dm2.data_ptr(), 0, dx.data_ptr(),
                                           dy.data_ptr(), n, batch, epochs, perm=dperm.data_ptr(), lr=lr)
    p = [np.asarray(a, np.float64) for a in params]
    m = [np.zeros_like(a) for a in p]
    v = [np.zeros_like(a) for a in p]
    step, ref_losses = 0, []
    for e in range(epochs):
        el = []
        for r0 in range(0, n, batch):
            idx = perm[e, r0:r0 + batch]
            el.append(OP.loss(p, x[idx], y[idx]))
            step += 1
            p, m, v = OP.adam_step(p, OP.grad(p, x[idx], y[idx]), m, v, step, lr=lr)
        ref_losses.append(np.mean(el))
    assert t == step == epochs * ((n + batch - 1) // batch)
    errs = [O.normwise_err(dp.cpu().numpy(), _flat(p)), O.normwise_err(dm1.cpu().numpy(), _flat(m)),
            O.normwise_err(dm2.cpu().numpy(), _flat(v))]
    log(f"  train loop vs oracle after {step} steps: params/m1/m2 err {errs[0]:.2e} {errs[1]:.2e} {errs[2]:.2e}")
    assert max(errs) <= 1e-5
    assert O.normwise_err(np.asarray(losses), np.asarray(ref_losses)) <= 1e-5
