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


def test_olsen_hand_example_and_closed_forms():
    # q_r = (1, 1), q_x = (0.6, -0.8), x.q_r = 1.4, x.q_x = -0.28: t = q_r + 5 q_x
    t = precond.olsen_candidate(np.array([0.6, 0.8]), np.array([1.0, -1.0]), np.array([1.0, 3.0]), 2.0)
    assert np.abs(t - np.array([4.0, -3.0])).max() < 1e-14
    rng = np.random.default_rng(6)
    n = 20
    H = rng.normal(size=(n, n))
    H = H + H.T
    x = rng.normal(size=n)
    x /= np.linalg.norm(x)
    theta = x @ H @ x
    r = H @ x - theta * x
    t = precond.olsen_candidate(x, r, np.diag(H).copy(), theta)
    assert abs(x @ t) < 1e-12 * np.linalg.norm(t)
    # constant diagonal c: t = (r - (x.r) x) / (theta - c) for any r
    r2 = rng.normal(size=n)
    t = precond.olsen_candidate(x, r2, np.full(n, 3.5), 1.25)
    assert np.abs(t - (r2 - (x @ r2) * x) / (1.25 - 3.5)).max() < 1e-13


def _pcg_case(seed, n=8):
    rng = np.random.default_rng(seed)
    H = rng.normal(size=(n, n))
    H = H + H.T + np.diag(rng.uniform(0, 4, size=n))
    x = rng.normal(size=n)
    x /= np.linalg.norm(x)
    Q = np.linalg.qr(np.column_stack([x, rng.normal(size=(n, n - 1))]))[0][:, 1:]  # complement of x
    lo = min(np.linalg.eigvalsh(Q.T @ H @ Q)[0], np.diag(H).min())
    theta = lo - 0.5  # theta - H negative definite on the complement, theta - d < 0
    r = H @ x - theta * x
    return H, x, Q, theta, r


def test_shift_invert_full_krylov_solves_the_projected_system():
    for seed in range(3):
        H, x, Q, theta, r = _pcg_case(seed)
        n = x.size
        t, mv = precond.shift_invert_candidate(lambda v: H @ v, x, r, np.diag(H).copy(), theta,
                                               steps=n - 1, rtol=0.0)
        ref = Q @ np.linalg.solve(Q.T @ (theta * np.eye(n) - H) @ Q, Q.T @ r)
        assert np.linalg.norm(t - ref) <= 1e-9 * np.linalg.norm(ref), seed
        assert abs(x @ t) <= 1e-12 * np.linalg.norm(t)
        assert mv <= n - 1


def test_shift_invert_steps_are_galerkin_over_the_krylov_space():
    """After j steps, t is the Galerkin solution of P (theta - H) P t = P r over
    span{z, (M A) z, ..., (M A)^{j-1} z} (z = M P r, M the projected diagonal
    inverse), built here column by column: the energy-norm minimiser."""
    H, x, Q, theta, r = _pcg_case(7, n=10)
    n = x.size
    d = np.diag(H).copy()
    P = np.eye(n) - np.outer(x, x)
    A = P @ (theta * np.eye(n) - H) @ P
    Mi = P @ np.diag(1.0 / (theta - d)) @ P
    b = P @ r
    for j in (1, 2, 3):
        cols = [Mi @ b]
        for _ in range(j - 1):
            cols.append(Mi @ (A @ cols[-1]))
        V = np.linalg.qr(np.column_stack(cols))[0]
        ref = V @ np.linalg.solve(V.T @ A @ V, V.T @ b)
        t, mv = precond.shift_invert_candidate(lambda v: H @ v, x, r, d, theta, steps=j, rtol=0.0)
        assert mv == j
        assert np.linalg.norm(t - ref) <= 1e-10 * np.linalg.norm(ref), j


def test_shift_invert_guard_returns_the_projected_diagonal():
    """theta above the spectrum: theta - H is positive definite, the first
    direction has non-negative curvature, and the projected diagonal
    correction is returned after one product."""
    H, x, Q, theta, r = _pcg_case(2)
    theta = np.linalg.eigvalsh(H)[-1] + 1.0
    r = H @ x - theta * x
    d = np.diag(H).copy()
    t, mv = precond.shift_invert_candidate(lambda v: H @ v, x, r, d, theta)
    P = np.eye(x.size) - np.outer(x, x)
    assert mv == 1
    assert np.abs(t - P @ (P @ r / (theta - d))).max() < 1e-13
