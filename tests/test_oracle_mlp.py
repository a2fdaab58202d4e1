"""Pins of the fp64 MLP reference: finite differences and a hand-derived Adam step."""
import numpy as np

from oracle import mlp


def test_mlp_gradient_finite_difference():
    rng = np.random.default_rng(0)
    P = mlp.init(5, 7, seed=1)
    for k in ("b1", "b2"):
        P[k] = rng.normal(0, 0.3, P[k].shape)  # move kinks away from the samples
    X = rng.normal(size=(11, 5))
    T = rng.normal(size=11)

    def loss(P):
        y, _ = mlp.forward(P, X)
        return mlp.cosine_loss(y, T)[0]

    y, cache = mlp.forward(P, X)
    _, dy = mlp.cosine_loss(y, T)
    G = mlp.backward(P, cache, dy)
    eps = 1e-6
    for k in mlp.PARAM_NAMES:
        for idx in [tuple(rng.integers(0, s) for s in P[k].shape) for _ in range(4)]:
            Pp = {kk: v.copy() for kk, v in P.items()}
            Pm = {kk: v.copy() for kk, v in P.items()}
            Pp[k][idx] += eps
            Pm[k][idx] -= eps
            fd = (loss(Pp) - loss(Pm)) / (2 * eps)
            assert abs(fd - G[k][idx]) < 1e-7, (k, idx, fd, G[k][idx])


def test_cosine_loss_scale_invariant():
    rng = np.random.default_rng(1)
    y, t = rng.normal(size=(2, 9))
    assert abs(mlp.cosine_loss(y, t)[0] - mlp.cosine_loss(3.7 * y, t)[0]) < 1e-14
    assert abs(mlp.cosine_loss(t, t)[0]) < 1e-14


def test_adam_first_step_is_signed_lr():
    # after one step from zero moments, the bias-corrected update is lr * g/(|g| + eps')
    P = {k: np.zeros(3) for k in mlp.PARAM_NAMES}
    G = {k: np.array([2.0, -0.5, 0.0]) for k in mlp.PARAM_NAMES}
    st = {}
    mlp.adam_step(P, G, st, lr=0.1)
    assert np.allclose(P["W1"], [-0.1, 0.1, 0.0], atol=1e-7)
