"""fp64 reference of the preconditioner network: a 3-layer ReLU MLP F -> H -> H -> 1.

y = W3 relu(W2 relu(W1 x + b1) + b2) + b3, applied row-wise to X[n, F].
Backward is the chain rule written out; Adam is the Kingma-Ba update
(m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2, bias-corrected step).
The per-triple loss is 1 - cos(delta, Delta) over the amplitudes of one
Davidson correction (the correction's scale is irrelevant to Davidson).

Pins: finite differences of the loss (``tests/test_oracle_mlp.py``).
"""
from __future__ import annotations

import numpy as np

PARAM_NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


def init(n_in, width, seed=0):
    rng = np.random.default_rng(seed)
    return {
        "W1": rng.normal(0, np.sqrt(2.0 / n_in), (width, n_in)),
        "b1": np.zeros(width),
        "W2": rng.normal(0, np.sqrt(2.0 / width), (width, width)),
        "b2": np.zeros(width),
        "W3": rng.normal(0, np.sqrt(1.0 / width), (1, width)),
        "b3": np.zeros(1),
    }


def forward(P, X):
    z1 = X @ P["W1"].T + P["b1"]
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ P["W2"].T + P["b2"]
    a2 = np.maximum(z2, 0.0)
    y = a2 @ P["W3"].T + P["b3"]
    return y[:, 0], (X, z1, a1, z2, a2)


def backward(P, cache, dy):
    X, z1, a1, z2, a2 = cache
    dy = dy[:, None]
    g = {"W3": dy.T @ a2, "b3": dy.sum(0)}
    da2 = dy @ P["W3"]
    dz2 = da2 * (z2 > 0)
    g["W2"] = dz2.T @ a1
    g["b2"] = dz2.sum(0)
    da1 = dz2 @ P["W2"]
    dz1 = da1 * (z1 > 0)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(0)
    return g


def cosine_loss(y, target):
    """1 - <y, t>/(|y||t|) and its gradient with respect to y."""
    ny = np.linalg.norm(y)
    nt = np.linalg.norm(target)
    c = float(y @ target) / (ny * nt)
    dy = target / (ny * nt) - c * y / (ny * ny)
    return 1.0 - c, -dy


def adam_step(P, G, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in PARAM_NAMES:
        m = state.setdefault("m_" + k, np.zeros_like(P[k]))
        v = state.setdefault("v_" + k, np.zeros_like(P[k]))
        m[...] = beta1 * m + (1 - beta1) * G[k]
        v[...] = beta2 * v + (1 - beta2) * G[k] ** 2
        mh = m / (1 - beta1 ** t)
        vh = v / (1 - beta2 ** t)
        P[k] = P[k] - lr * mh / (np.sqrt(vh) + eps)
    return P
