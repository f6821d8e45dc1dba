"""Plain numpy float64 oracle of the triage network (test infrastructure).

The network scores (kernel, seed) instances for race likelihood:
  h1 = relu(X W1^T + b1), h2 = relu(h1 W2^T + b2), z = h2 w3 + b3,
trained with the mean binary cross-entropy on logits, softplus(z) - y z,
by Adam (Kingma and Ba 2015: beta1 = 0.9, beta2 = 0.999, eps = 1e-8, bias
corrections 1 - beta^t).  Gradients are written out by the chain rule.

Parameters are one flat float vector in this order:
  W1 [256 x 128], b1 [256], W2 [256 x 256], b2 [256], w3 [256], b3 [1]
(99,073 values).  Only tests and the benchmark's reference leg use this file.
"""
from __future__ import annotations

import numpy as np

D_IN, D_H = 128, 256
SHAPES = [("W1", (D_H, D_IN)), ("b1", (D_H,)), ("W2", (D_H, D_H)), ("b2", (D_H,)), ("w3", (D_H,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)
ADAM_B1, ADAM_B2, ADAM_EPS = 0.9, 0.999, 1e-8


def unpack(theta: np.ndarray) -> dict:
    out, at = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = theta[at:at + n].reshape(shape)
        at += n
    return out


def pack(parts: dict) -> np.ndarray:
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def forward(theta: np.ndarray, X: np.ndarray):
    p = unpack(np.asarray(theta, dtype=np.float64))
    X = np.asarray(X, dtype=np.float64)
    a1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ p["w3"] + p["b3"][0]
    return z, (X, a1, h1, a2, h2)


def softplus(z):
    return np.logaddexp(0.0, z)


def loss(theta, X, y) -> float:
    z, _ = forward(theta, X)
    y = np.asarray(y, dtype=np.float64)
    return float(np.mean(softplus(z) - y * z))


def grad(theta, X, y):
    """Gradient of the mean loss with respect to every parameter, and the loss."""
    p = unpack(np.asarray(theta, dtype=np.float64))
    z, (X, a1, h1, a2, h2) = forward(theta, X)
    y = np.asarray(y, dtype=np.float64)
    n = X.shape[0]
    sig = 1.0 / (1.0 + np.exp(-z))
    dz = (sig - y) / n                     # d mean(softplus(z) - y z) / dz
    g = {"w3": h2.T @ dz, "b3": np.array([dz.sum()])}
    dh2 = np.outer(dz, p["w3"])
    da2 = dh2 * (a2 > 0)
    g["W2"] = da2.T @ h1
    g["b2"] = da2.sum(axis=0)
    dh1 = da2 @ p["W2"]
    da1 = dh1 * (a1 > 0)
    g["W1"] = da1.T @ X
    g["b1"] = da1.sum(axis=0)
    return pack(g), float(np.mean(softplus(z) - y * z))


def adam_step(theta, m, v, g, step: int, lr: float):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = ADAM_B1 * m + (1 - ADAM_B1) * g
    v = ADAM_B2 * v + (1 - ADAM_B2) * g * g
    mhat = m / (1 - ADAM_B1 ** step)
    vhat = v / (1 - ADAM_B2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + ADAM_EPS), m, v
