"""Test infrastructure only (never imported by the library): fp64 reference of
the Davidson correction candidates of the learned preconditioner.

Diagonal (Davidson-Jacobi) candidate, per amplitude:
    t_i = r_i / (theta - d_i),  |theta - d_i| floored at 1e-8 (sign kept).

Per-amplitude features of the learned candidate (8 scale-free numbers; the
network maps them to the correction delta_i).  A "block" is one dense block
of the two-site vector (left sector, physical pair, right sector); e = d - theta:
    f0  r_i sqrt(n) / |r|
    f1  e_i / s_b               s_b = mean over the block of |e| (floored at 1e-300)
    f2  clip(s_b / e_i, -10, 10)   (e_i = 0 gives +10)
    f3  t_i sqrt(n) / |t|       the diagonal candidate, normalised
    f4  mean over the block of e / s_b
    f5  min over the block of e / s_b
    f6  log(block size) / 10
    f7  k / L                   position of the two-site step on the chain
Invariances (pinned in tests): scaling r by a only multiplies f0 and f3 by
sign(a) and leaves the rest unchanged; f1, f2, f4, f5 do not change when H is
scaled and shifted (d, theta -> a d + b, a theta + b with a > 0).

The paper gives no formula for these features (it names a run-time-selectable
preconditioner family, not a learned member), so this module is their
definition; it is pinned by the invariances above and a hand-computed example
(tests/test_oracle_precond.py).

The other members of that family (Sec. III names Jacobi, the deflation-aware
diagonal, Olsen and a shift-and-invert inner-PCG mode with an indefiniteness
guard) are written here from their textbook definitions, since the paper
states only their names:
  Olsen:  t = q_r - (x.q_r / x.q_x) q_x, q_v = (theta - d)^-1 v (floored as
          above), x the unit Ritz vector and r = (H - theta) x its residual;
  shift-and-invert: the Jacobi-Davidson correction equation
          P (theta - H) P t = P r,  P = 1 - x x^T,  t orthogonal to x,
          solved approximately by preconditioned conjugate gradients with the
          projected diagonal P (theta - d)^-1 as preconditioner.  Near the
          lowest root both operators are negative definite on the complement
          of x and CG runs as on their negatives.  The guard: an iteration
          whose curvature p.A p is not negative (or whose rho = res.z is not
          negative) stops; stopping at the first iteration returns the
          projected diagonal correction.  Otherwise at most `steps`
          iterations, ending early once |res| <= rtol |r|.
Pins (tests/test_oracle_precond.py): x.t = 0 and the constant-diagonal
closed form for Olsen; for the PCG, the exact solution of the projected
system at full Krylov dimension, the Galerkin (energy-norm) minimiser over the
explicitly built preconditioned Krylov space after 1-3 steps, and the guard
on a positive definite shift.
"""
from __future__ import annotations

import numpy as np

N_FEATURES = 8


def diag_candidate(r, d, theta):
    den = theta - d
    small = np.abs(den) < 1e-8
    den = np.where(small, np.where(den < 0, -1e-8, 1e-8), den)
    return r / den


def features(r, d, theta, blocks, k, L):
    """blocks: list of index arrays (flat positions of each block's amplitudes)."""
    n = r.size
    e = d - theta
    t = diag_candidate(r, d, theta)
    X = np.zeros((n, N_FEATURES))
    X[:, 0] = r * np.sqrt(n) / np.linalg.norm(r)
    X[:, 3] = t * np.sqrt(n) / np.linalg.norm(t)
    X[:, 7] = k / L
    for idx in blocks:
        eb = e[idx]
        s = max(np.mean(np.abs(eb)), 1e-300)
        u = eb / s
        X[idx, 1] = u
        with np.errstate(divide="ignore"):
            inv = np.where(eb == 0, 10.0, s / np.where(eb == 0, 1.0, eb))
        X[idx, 2] = np.clip(inv, -10.0, 10.0)
        X[idx, 4] = np.mean(u)
        X[idx, 5] = np.min(u)
        X[idx, 6] = np.log(idx.size) / 10.0
    return X


def projected_target(psi_i, psi_star):
    """Delta = P_perp psi* (P_perp projects out the normalised psi_i), with psi*
    oriented so that <psi_i, psi*> >= 0."""
    p = psi_i / np.linalg.norm(psi_i)
    c = float(p @ psi_star)
    s = psi_star if c >= 0 else -psi_star
    return s - abs(c) * p


def olsen_candidate(x, r, d, theta):
    """Olsen's correction: the diagonal correction less its component along
    (theta - d)^-1 x, so that x.t = 0."""
    qr = diag_candidate(r, d, theta)
    qx = diag_candidate(x, d, theta)
    return qr - (x @ qr) / (x @ qx) * qx


def shift_invert_candidate(apply, x, r, d, theta, steps=5, rtol=0.1):
    """Approximate solution of P (theta - H) P t = P r by preconditioned CG
    (apply(v) = H v).  Returns (t, number of H products)."""
    def proj(v):
        return v - (x @ v) * x

    def A(v):  # P (theta - H) P on vectors already orthogonal to x
        return proj(theta * v - apply(v))

    def Minv(v):
        return proj(diag_candidate(v, d, theta))

    rnorm = np.linalg.norm(r)
    t = np.zeros_like(r)
    res = proj(r)
    z = Minv(res)
    rho = res @ z
    p = z.copy()
    products = 0
    for j in range(steps):
        q = A(p)
        products += 1
        curv = p @ q
        if not (curv < 0 and rho < 0):
            if j == 0:
                t = z.copy()
            break
        alpha = rho / curv
        t = t + alpha * p
        res = res - alpha * q
        if j + 1 == steps or np.linalg.norm(res) <= rtol * rnorm:
            break
        z = Minv(res)
        rho_new = res @ z
        p = z + (rho_new / rho) * p
        rho = rho_new
    return t, products
