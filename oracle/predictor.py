"""FP64 learned contention predictor: forward, backward and Adam (test infrastructure).

The paper predicts each microservice's duration from its batch size and compute
share with offline-trained models (Section VII-A, where a decision tree is chosen
among linear regression, decision tree and random forest). The learned
predictor here replaces that model with a small MLP
    16 -> 64 (ReLU) -> 64 (ReLU) -> 1 (linear)
that maps a stage's share, batch and co-runner features to ln(latency).
Weights are [in, out] row-major, biases per output.

Loss: L = (1/M) sum_r (yhat_r - y_r)^2 over a minibatch of M rows.
Adam: Kingma & Ba (2015), bias-corrected moments, beta1 0.9, beta2 0.999,
eps 1e-8.

Pinned (tests/test_oracle_misc.py) by central finite differences of the loss, by
Adam's first step (lr * sign(g) up to eps), and by hand-derived values of the
second and third steps for scalar gradient sequences (g = 1 then -1: the second
bias-corrected second moment is exactly 1 and the step is -lr/19; g = 1 then 0:
the step is lr * (9/19) / sqrt(999/1999)), which fix beta1, beta2 and both bias
corrections beyond t = 1.
"""
from __future__ import annotations

import numpy as np

DIMS = (16, 64, 64, 1)


def _f64(params):
    return [np.asarray(p, np.float64) for p in params]


def forward(params, x):
    """Returns (yhat [M], cache)."""
    w1, b1, w2, b2, w3, b3 = _f64(params)
    x = np.asarray(x, np.float64)
    z1 = x @ w1 + b1
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ w2 + b2
    a2 = np.maximum(z2, 0.0)
    yhat = (a2 @ w3 + b3)[:, 0]
    return yhat, (x, z1, a1, z2, a2)


def loss(params, x, y) -> float:
    yhat, _ = forward(params, x)
    d = yhat - np.asarray(y, np.float64)
    return float(np.mean(d * d))


def grad(params, x, y):
    """Gradients of the loss w.r.t. [w1, b1, w2, b2, w3, b3] (FP64)."""
    w1, b1, w2, b2, w3, b3 = _f64(params)
    yhat, (x, z1, a1, z2, a2) = forward(params, x)
    m = x.shape[0]
    dy = 2.0 * (yhat - np.asarray(y, np.float64)) / m        # [M]
    gw3 = a2.T @ dy[:, None]
    gb3 = np.array([dy.sum()])
    dz2 = (dy[:, None] @ w3.T) * (z2 > 0)
    gw2 = a1.T @ dz2
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ w2.T) * (z1 > 0)
    gw1 = x.T @ dz1
    gb1 = dz1.sum(axis=0)
    return [gw1, gb1, gw2, gb2, gw3, gb3]


def adam_step(params, grads, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t (1-based). Returns (params, m, v), all FP64."""
    out_p, out_m, out_v = [], [], []
    for p, g, mi, vi in zip(_f64(params), _f64(grads), _f64(m), _f64(v)):
        mi = beta1 * mi + (1 - beta1) * g
        vi = beta2 * vi + (1 - beta2) * g * g
        mhat = mi / (1 - beta1 ** t)
        vhat = vi / (1 - beta2 ** t)
        out_p.append(p - lr * mhat / (np.sqrt(vhat) + eps))
        out_m.append(mi)
        out_v.append(vi)
    return out_p, out_m, out_v


def numeric_grad(params, x, y, h=1e-6):
    """Central differences of the loss for every parameter (slow; small inputs)."""
    ps = _f64(params)
    out = []
    for i, p in enumerate(ps):
        g = np.zeros_like(p)
        it = np.nditer(p, flags=["multi_index"])
        for _ in it:
            idx = it.multi_index
            old = p[idx]
            p[idx] = old + h
            lp = loss(ps, x, y)
            p[idx] = old - h
            lm = loss(ps, x, y)
            p[idx] = old
            g[idx] = (lp - lm) / (2 * h)
        out.append(g)
    return out
