"""Pins of the oracle's preconditioner candidates: a hand-computed example and
the invariances that make the features scale-free."""
import numpy as np

from oracle import precond


def test_features_hand_example():
    r = np.array([1.0, -2.0, 0.5, 4.0])
    d = np.array([3.0, 1.5, 2.0, 0.0])
    blocks = [np.array([0, 1]), np.array([2, 3])]
    X = precond.features(r, d, 1.0, blocks, 2, 8)
    nr, nt = np.sqrt(21.25), np.sqrt(32.5)
    expect = np.array([
        [2 * 1.0 / nr, 1.6, 0.625, 2 * -0.5 / nt, 1.0, 0.4, np.log(2) / 10, 0.25],
        [2 * -2.0 / nr, 0.4, 2.5, 2 * 4.0 / nt, 1.0, 0.4, np.log(2) / 10, 0.25],
        [2 * 0.5 / nr, 1.0, 1.0, 2 * -0.5 / nt, 0.0, -1.0, np.log(2) / 10, 0.25],
        [2 * 4.0 / nr, -1.0, -1.0, 2 * 4.0 / nt, 0.0, -1.0, np.log(2) / 10, 0.25],
    ])
    assert np.abs(X - expect).max() < 1e-14


def test_diag_candidate_floor_and_zero_gap_feature():
    t = precond.diag_candidate(np.array([1.0, 1.0]), np.array([2.0, 2.0 + 1e-12]), 2.0)
    assert t[0] == 1e8 and t[1] == -1e8
    X = precond.features(np.array([1.0, 2.0]), np.array([2.0, 3.0]), 2.0, [np.array([0, 1])], 0, 4)
    assert X[0, 2] == 10.0 and X[0, 1] == 0.0


def test_feature_invariances():
    rng = np.random.default_rng(3)
    n = 60
    r, d = rng.normal(size=n), rng.normal(size=n) + 2
    blocks = [np.arange(0, 10), np.arange(10, 35), np.arange(35, 60)]
    X = precond.features(r, d, 0.3, blocks, 3, 10)
    Xr = precond.features(-2.5 * r, d, 0.3, blocks, 3, 10)
    Xh = precond.features(r, 3.0 * d - 1.0, 3.0 * 0.3 - 1.0, blocks, 3, 10)
    assert np.abs(X[:, 0] + Xr[:, 0]).max() < 1e-13
    assert np.abs(X[:, 3] + Xr[:, 3]).max() < 1e-13
    assert np.abs(X[:, [1, 2, 4, 5, 6, 7]] - Xr[:, [1, 2, 4, 5, 6, 7]]).max() < 1e-13
    assert np.abs(X[:, [1, 2, 4, 5]] - Xh[:, [1, 2, 4, 5]]).max() < 1e-12
    # per-block constants
    for b in blocks:
        assert np.ptp(X[b, 4]) == 0 and np.ptp(X[b, 5]) == 0 and np.ptp(X[b, 6]) == 0


def test_projected_target():
    rng = np.random.default_rng(4)
    p, s = rng.normal(size=(2, 30))
    D = precond.projected_target(p, s)
    assert abs(D @ p) < 1e-12 * np.linalg.norm(p) * np.linalg.norm(s)
    D2 = precond.projected_target(p, -s)
    assert np.abs(D - D2).max() < 1e-14  # orientation fixed by <psi_i, psi*> >= 0
    q = np.zeros(30)
    q[0] = 1.0
    s0 = s.copy()
    s0[0] = 0.0
    assert np.abs(precond.projected_target(q, s0) - s0).max() < 1e-15
