"""Orbital entanglement for the ordering of the chain.  TEST INFRASTRUCTURE ONLY
(see ``oracle/__init__.py``).

Sec. II.H orders the lattice by the pairwise mutual information I_ij of the
orbitals (the Fiedler vector of its graph Laplacian) and cites the orbital
entanglement of Legeza and Rissler; the definitions below are those standard
ones, written from their statements:

* one- and two-orbital reduced density matrices: with the spin orbitals of
  orbital i (or of i < j) moved to the front of the creator string, in the
  local order (i alpha, j alpha, i beta, j beta), a determinant is
  +-|local> x |env>; rho = Tr_env |Psi><Psi| / <Psi|Psi>.  Local states are
  s = n_alpha + 2 n_beta per orbital and, for a pair, L = s_i + 4 s_j;
* s_i = -sum p ln p over the eigenvalues of rho_i (natural log), s_ij likewise;
* I_ij = (s_i + s_j - s_ij) / 2 for i != j, I_ii = 0;
* ordering: the eigenvector of the second-smallest eigenvalue of
  L = diag(sum_j I_ij) - I, its sign fixed so that the component of largest
  magnitude (first such index) is positive; orbitals sorted by ascending
  component (stable sort).

The move of the local creators to the front is done here by counting
inversions of the permuted creator string (brute force).  Pins
(``tests/test_oracle_orbital.py``): expectation values of |t><s| built from
brute-force Fock-space ladder operators, a determinant (no entanglement), the
two-orbital singlet (s_i = ln 2, s_ij = 0), traces and partial traces, and
the Fiedler vector of a path graph.
"""
from __future__ import annotations

import numpy as np

from . import fci


def _perm_parity(seq):
    inv = 0
    for a in range(len(seq)):
        for b in range(a + 1, len(seq)):
            inv += seq[a] > seq[b]
    return -1.0 if inv & 1 else 1.0


def _local_order(n, orbs):
    """Spin-orbital positions (alpha-first order: p, n + p) of the local orbitals,
    all alphas then all betas, orbitals in the given order."""
    return [p for p in orbs] + [n + p for p in orbs]


def orbital_rdm(space: fci.DetSpace, C: np.ndarray, orbs):
    """rho over the local states of `orbs` (one orbital: 4 states, two: 16)."""
    n = space.n
    C = C.reshape(space.shape)
    loc = _local_order(n, orbs)
    dim = 4 ** len(orbs)
    groups = {}
    for ia, a in enumerate(space.sa):
        for ib, b in enumerate(space.sb):
            amp = C[ia, ib]
            bits = int(a) | (int(b) << n)
            occ = [x for x in range(2 * n) if bits >> x & 1]  # creator string, alpha-first order
            local = [x for x in loc if bits >> x & 1]
            env = [x for x in occ if x not in loc]
            # the creator string reordered to local (local order) + env: its parity
            sign = _perm_parity([occ.index(x) for x in local + env])
            L = 0
            for t, p in enumerate(orbs):
                s = (bits >> p & 1) + 2 * (bits >> (n + p) & 1)
                L += s * 4 ** t
            envkey = tuple(env)
            groups.setdefault(envkey, np.zeros(dim))[L] += sign * amp
    rho = sum(np.outer(v, v) for v in groups.values())
    return rho / float(np.sum(C * C))


def entropy(rho):
    w = np.linalg.eigvalsh(rho)
    w = w[w > 1e-300]
    return float(-np.sum(w * np.log(w)))


def mutual_information(space, C):
    n = space.n
    s1 = np.array([entropy(orbital_rdm(space, C, [i])) for i in range(n)])
    I = np.zeros((n, n))
    for i in range(n):
        for j in range(i + 1, n):
            I[i, j] = I[j, i] = 0.5 * (s1[i] + s1[j] - entropy(orbital_rdm(space, C, [i, j])))
    return s1, I


def fiedler_order(I):
    Lap = np.diag(I.sum(axis=1)) - I
    w, V = np.linalg.eigh(Lap)
    v = V[:, 1]
    k = int(np.argmax(np.abs(v)))
    if v[k] < 0:
        v = -v
    return np.argsort(v, kind="stable"), v
