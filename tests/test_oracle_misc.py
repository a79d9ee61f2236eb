"""Pins of the oracle's delivery check, statistics and predictor."""
import os

import numpy as np

from oracle import delivery as D
from oracle import predictor as P
from oracle import stats as S
import workload_gen as G

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- splitmix64
def test_splitmix64_published_outputs():
    with open(os.path.join(GOLDEN, "splitmix64.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    assert rows
    for row in rows:
        state = int(row[0])
        for want in row[1:]:
            state, out = D.splitmix64_next(state)
            assert out == int(want)
    assert D.id_hash(0) == 0xE220A8397B1DCDAF


def test_checksum_algebra():
    a = list(range(100, 150))
    b = list(range(150, 170))
    sa, xa = D.checksums(a)
    sb, xb = D.checksums(b)
    s, x = D.checksums(a + b)
    assert s == (sa + sb) % (1 << 64) and x == xa ^ xb
    # order independence and xor cancellation of a duplicate
    assert D.checksums(reversed(a)) == (sa, xa)
    assert D.checksums(a + [a[0]])[1] == xa ^ D.id_hash(a[0])


def test_delivery_check_detects_problems():
    sub = list(range(10))
    assert D.check_delivery(sub, sub) == []
    assert any("lost" in p for p in D.check_delivery(sub, sub[:-1]))
    assert any("duplicated" in p for p in D.check_delivery(sub, sub + [3]))
    assert any("order" in p for p in D.check_delivery(sub, [1, 0] + sub[2:]))
    assert any("unknown" in p for p in D.check_delivery(sub, sub + [99]))


# ---------------------------------------------------------------- stats
def test_nearest_rank():
    v = list(range(1, 101))
    assert S.nearest_rank(v, 0.99) == 99
    assert S.nearest_rank(v, 0.5) == 50
    assert S.nearest_rank(v, 1.0) == 100
    assert S.nearest_rank([7], 0.99) == 7
    # definition by counting, on a shuffled sample with repeats
    g = G.rng("handoff", 21)
    w = list(g.integers(0, 30, 57))
    for q in (0.1, 0.5, 0.9, 0.99):
        r = S.nearest_rank(w, q)
        assert sum(1 for t in w if t <= r) >= q * len(w)
        assert sum(1 for t in w if t < r) < q * len(w)


def test_latency_identity():
    assert S.check_latency_identity(0, [5, 20], [15, 30], 31)
    assert not S.check_latency_identity(0, [5, 12], [15, 30], 31)   # overlap -> negative queue
    q, s, g = S.latency_terms(100, [110], [150], 160)
    assert (q, s, g) == ([10], [40], 10)


# ---------------------------------------------------------------- predictor
def _small_problem():
    params = G.predictor_init(seed=4)
    x, y = G.predictor_batch(8, seed=4)
    return params, x, y


def test_predictor_grad_matches_finite_differences():
    params, x, y = _small_problem()
    # move biases off zero so ReLU kinks are not hit by the +-h probes
    params = [p + 0.01 * (i % 2) for i, p in enumerate(params)]
    g = P.grad(params, x, y)
    n = P.numeric_grad(params, x, y)
    for a, b in zip(g, n):
        assert a.shape == np.asarray(b).shape
        assert np.max(np.abs(a - b)) <= 1e-5 * max(1.0, np.max(np.abs(b)))


def test_predictor_adam_first_step_is_lr_sign():
    params, x, y = _small_problem()
    g = P.grad(params, x, y)
    zeros = [np.zeros_like(np.asarray(p, np.float64)) for p in params]
    newp, m, v = P.adam_step(params, g, zeros, zeros, t=1, lr=1e-3)
    for p0, p1, gi in zip(params, newp, g):
        step = np.asarray(p1) - np.asarray(p0, np.float64)
        big = np.abs(gi) > 1e-4
        assert np.allclose(step[big], -1e-3 * np.sign(gi[big]), rtol=1e-3)


def _adam_scalar(gs, lr=0.1):
    p, m, v = [np.zeros(1)], [np.zeros(1)], [np.zeros(1)]
    for t, g in enumerate(gs, start=1):
        p, m, v = P.adam_step(p, [np.array([g], np.float64)], m, v, t, lr=lr)
    return p[0][0], m[0][0], v[0][0]


def test_predictor_adam_later_steps_hand_derived():
    """Kingma & Ba with beta1 = 0.9, beta2 = 0.999, eps = 1e-8, worked by hand for
    scalar gradient sequences from zero moments, lr = 0.1.

    g = (1, -1): m2 = 0.9 * 0.1 - 0.1 = -0.01, v2 = 0.999 * 0.001 + 0.001 = 0.001999;
    the corrected moments are -0.01 / 0.19 = -1/19 and 0.001999 / 0.001999 = 1, so
    the second step is +0.1 / 19 / (1 + eps) after a first step of -0.1 / (1 + eps).
    g = (1, 0): m2 = 0.09, v2 = 0.000999, corrected 9/19 and 999/1999.
    g = (1, 0, 0): m3 = 0.081, v3 = 0.000998001, corrected 0.081 / 0.271 = 81/271 and
    0.000998001 / 0.002997001 = 998001/2997001."""
    eps = 1e-8
    first = -0.1 / (1 + eps)
    p, m, v = _adam_scalar([1.0, -1.0])
    assert np.isclose(m, -0.01, rtol=1e-12, atol=0) and np.isclose(v, 0.001999, rtol=1e-12, atol=0)
    assert np.isclose(p, first + 0.1 / 19 / (1 + eps), rtol=1e-12, atol=0)
    p, m, v = _adam_scalar([1.0, 0.0])
    assert np.isclose(m, 0.09, rtol=1e-12, atol=0) and np.isclose(v, 0.000999, rtol=1e-12, atol=0)
    step2 = 0.1 * (9 / 19) / (np.sqrt(999 / 1999) + eps)
    assert np.isclose(p, first - step2, rtol=1e-12, atol=0)
    p, m, v = _adam_scalar([1.0, 0.0, 0.0])
    assert np.isclose(m, 0.081, rtol=1e-12, atol=0) and np.isclose(v, 0.000998001, rtol=1e-12, atol=0)
    step3 = 0.1 * (81 / 271) / (np.sqrt(998001 / 2997001) + eps)
    assert np.isclose(p, first - step2 - step3, rtol=1e-12, atol=0)
    # the numbers themselves, written out (9/19 = 0.47368..., sqrt(999/1999) = 0.70693...)
    assert abs(step2 - 0.067005816) < 1e-8


def test_predictor_training_reduces_loss():
    params, x, y = _small_problem()
    m = [np.zeros_like(np.asarray(p, np.float64)) for p in params]
    v = [np.zeros_like(np.asarray(p, np.float64)) for p in params]
    l0 = P.loss(params, x, y)
    p = params
    for t in range(1, 201):
        p, m, v = P.adam_step(p, P.grad(p, x, y), m, v, t, lr=1e-2)
    assert P.loss(p, x, y) < 0.1 * l0
