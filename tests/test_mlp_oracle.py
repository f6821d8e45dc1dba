"""Pins of the triage network's numpy oracle (oracle/mlp.py).

The oracle's gradient is written out by hand, so it is pinned to things that
do not share that derivation: central finite differences of the loss, torch's
float64 autograd on the same network, and closed forms for the special cases
(output bias only, zero logits, the first Adam step).
"""
import math

import numpy as np
import pytest

from oracle import mlp as M


def _init(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    parts = {
        "W1": rng.normal(0, scale / math.sqrt(M.D_IN), (M.D_H, M.D_IN)),
        "b1": rng.normal(0, 0.1, M.D_H),
        "W2": rng.normal(0, scale / math.sqrt(M.D_H), (M.D_H, M.D_H)),
        "b2": rng.normal(0, 0.1, M.D_H),
        "w3": rng.normal(0, 1 / math.sqrt(M.D_H), M.D_H),
        "b3": rng.normal(0, 0.1, 1),
    }
    return M.pack(parts)


def _data(seed, n):
    rng = np.random.default_rng(seed)
    X = rng.normal(0, 1, (n, M.D_IN))
    y = (rng.random(n) < 0.4).astype(np.float64)
    return X, y


def test_param_count():
    assert M.N_PARAMS == 128 * 256 + 256 + 256 * 256 + 256 + 256 + 1 == 99073
    theta = np.arange(M.N_PARAMS, dtype=np.float64)
    assert np.array_equal(M.pack(M.unpack(theta)), theta)
    p = M.unpack(theta)
    assert p["W1"][1, 0] == 128 and p["b1"][0] == 128 * 256 and p["b3"][0] == M.N_PARAMS - 1


def test_gradient_central_differences():
    theta = _init(1)
    X, y = _data(2, 12)
    g, _ = M.grad(theta, X, y)
    rng = np.random.default_rng(3)
    # a sample from every parameter block, including both biases at the ends
    sizes = [int(np.prod(s)) for _, s in M.SHAPES]
    starts = np.cumsum([0] + sizes[:-1])
    idx = []
    for st, sz in zip(starts, sizes):
        idx += list(st + rng.choice(sz, size=min(sz, 40), replace=False))
    eps = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        fd = (M.loss(tp, X, y) - M.loss(tm, X, y)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(g[i]), 1e-3), (i, fd, g[i])


def test_gradient_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    theta = _init(4, scale=2.0)
    X, y = _data(5, 33)
    g, l = M.grad(theta, X, y)
    p = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in M.unpack(theta.copy()).items()}
    Xt, yt = torch.tensor(X), torch.tensor(y)
    h1 = torch.relu(Xt @ p["W1"].T + p["b1"])
    h2 = torch.relu(h1 @ p["W2"].T + p["b2"])
    z = h2 @ p["w3"] + p["b3"]
    lt = torch.nn.functional.binary_cross_entropy_with_logits(z, yt)
    lt.backward()
    gt = np.concatenate([p[k].grad.numpy().reshape(-1) for k, _ in M.SHAPES])
    assert abs(lt.item() - l) <= 1e-12
    assert np.max(np.abs(gt - g)) <= 1e-12 * max(1.0, np.max(np.abs(gt)))


def test_output_bias_only_closed_form():
    # w3 = 0: the logit is b3 for every row, loss = softplus(b3) - mean(y) b3,
    # d loss / d b3 = sigmoid(b3) - mean(y), and no other parameter gets gradient
    theta = _init(6)
    p = M.unpack(theta)
    p["w3"][:] = 0.0
    p["b3"][0] = 0.7
    X, y = _data(7, 20)
    z, _ = M.forward(theta, X)
    assert np.all(z == 0.7)
    g, l = M.grad(theta, X, y)
    ybar = y.mean()
    assert abs(l - (math.log1p(math.exp(0.7)) - ybar * 0.7)) < 1e-14
    assert abs(g[-1] - (1 / (1 + math.exp(-0.7)) - ybar)) < 1e-14
    gp = M.unpack(g)
    for k in ("W1", "b1", "W2", "b2"):
        assert np.all(gp[k] == 0.0)
    # gradient of w3 is the mean of h2 weighted by (sigmoid - y)
    _, (_, _, _, _, h2) = M.forward(theta, X)
    assert np.allclose(gp["w3"], h2.T @ ((1 / (1 + math.exp(-0.7)) - y) / len(y)), rtol=0, atol=1e-14)


def test_zero_first_layer_constant_hidden():
    # W1 = 0: every row has h1 = relu(b1), so every logit equals one hand-computed number
    theta = _init(8)
    p = M.unpack(theta)
    p["W1"][:] = 0.0
    X, _ = _data(9, 5)
    z, _ = M.forward(theta, X)
    h1 = [max(b, 0.0) for b in p["b1"]]
    expect = p["b3"][0]
    for j in range(M.D_H):
        a2 = p["b2"][j] + sum(p["W2"][j, i] * h1[i] for i in range(M.D_H))
        expect += max(a2, 0.0) * p["w3"][j]
    assert np.allclose(z, expect, rtol=0, atol=1e-12)


def test_zero_logit_loss_is_ln2():
    theta = np.zeros(M.N_PARAMS)
    X, y = _data(10, 9)
    assert abs(M.loss(theta, X, y) - math.log(2)) < 1e-15


def test_first_adam_step_closed_form():
    # step 1: bias-corrected moments are g and g^2, so the update is lr g / (|g| + eps)
    rng = np.random.default_rng(11)
    theta = rng.normal(size=50)
    g = rng.normal(size=50)
    g[0] = 0.0
    t1, m1, v1 = M.adam_step(theta, np.zeros(50), np.zeros(50), g, 1, 1e-3)
    assert np.allclose(t1, theta - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert t1[0] == theta[0]
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)
    # a constant gradient leaves the bias-corrected moments at g and g^2, so
    # every later step is the same lr g / (|g| + eps)
    m, v, t = m1, v1, t1
    for step in range(2, 6):
        t_new, m, v = M.adam_step(t, m, v, g, step, 1e-3)
        assert np.allclose(t - t_new, 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-14)
        t = t_new


def test_training_reduces_loss():
    theta = _init(12)
    rng = np.random.default_rng(13)
    X = rng.normal(size=(256, M.D_IN))
    y = (X[:, 0] + 0.5 * X[:, 1] > 0).astype(np.float64)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    l0 = M.loss(theta, X, y)
    for step in range(1, 41):
        g, _ = M.grad(theta, X, y)
        theta, m, v = M.adam_step(theta, m, v, g, step, 1e-3)
    l1 = M.loss(theta, X, y)
    assert l1 < 0.5 * l0
