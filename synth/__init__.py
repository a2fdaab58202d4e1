"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module only *makes inputs*: active-space integrals (h, B^Q) and random
block-sparse matrix-product states / two-site vectors in the documented storage
format.  It holds none of the method's arithmetic (no Hamiltonian application,
no contraction, no eigensolve), so importing it from both the oracle side and
the GPU side shares no computation between them.

Hamiltonian recipe (the paper factorises the two-electron integrals through
Cholesky vectors, (pq|rs) = sum_Q B^Q_pq B^Q_rs, Sec. II.A; the active space is
random because no molecule is used here):

1. h_pp = -2 + 3 p / (n - 1): a linear ramp from -2 to +1 Ha.
2. G = rng.normal(0, 0.05, (n, n)); h_pq = h_qp = G_pq for p < q
   (0.05 is a standard deviation).
3. C = rng.normal(0, 0.1, (n_chol, n, n)); B^Q_pq = B^Q_qp = C^Q_pq for p <= q.
4. E_core = 0.

Draw order is exactly 2 then 3 from one ``numpy.random.default_rng(seed)``.

Storage format of block-sparse tensors (shared convention with the C ABI):

* A bond at cut c (c orbitals to its left) is a list of sectors
  (N, 2S_z, dim) sorted ascending by (N, 2S_z).
* Site states s = 0..3 are |0>, |alpha>, |beta>, |alpha beta>, with quantum
  numbers (0,0), (1,+1), (1,-1), (2,0).
* A site tensor at site k is stored slab by slab: for each left sector q_l of
  bond k (in bond order) a row-major m_l x W matrix whose columns are the
  blocks s = 0..3 (those whose q_l + q_s is a sector of bond k+1) in s order,
  each m_r wide.
* A two-site vector at sites (k, k+1) uses the same slab form with a 16-valued
  physical index s = 4 s1 + s2 and right sectors taken from bond k+2.
"""
from __future__ import annotations

from math import comb

import numpy as np

SITE_QN = ((0, 0), (1, 1), (1, -1), (2, 0))


def make_hamiltonian(n: int, n_chol: int, seed: int = 0):
    """Return (h, B, e_core) for a CAS(n, n)-sized random active space."""
    rng = np.random.default_rng(seed)
    h = np.zeros((n, n))
    for p in range(n):
        h[p, p] = -2.0 + (3.0 * p / (n - 1) if n > 1 else 0.0)
    G = rng.normal(0.0, 0.05, (n, n))
    iu = np.triu_indices(n, 1)
    h[iu] = G[iu]
    h[(iu[1], iu[0])] = G[iu]
    C = rng.normal(0.0, 0.1, (n_chol, n, n))
    B = np.zeros((n_chol, n, n))
    iu0 = np.triu_indices(n, 0)
    for Q in range(n_chol):
        B[Q][iu0] = C[Q][iu0]
        B[Q][(iu0[1], iu0[0])] = C[Q][iu0]
    return h, B, 0.0


def full_bond_sectors(n: int, n_alpha: int, n_beta: int, cut: int):
    """All sectors (N, 2Sz, full_dim) at a cut with `cut` orbitals on the left.

    full_dim = min(#left states, #right states) for that split of electrons.
    """
    out = []
    for na in range(0, min(cut, n_alpha) + 1):
        for nb in range(0, min(cut, n_beta) + 1):
            ra, rb = n_alpha - na, n_beta - nb
            if ra > n - cut or rb > n - cut:
                continue
            left = comb(cut, na) * comb(cut, nb)
            right = comb(n - cut, ra) * comb(n - cut, rb)
            d = min(left, right)
            if d > 0:
                out.append((na + nb, na - nb, d))
    out.sort()
    return out


def bond_sectors(n: int, n_alpha: int, n_beta: int, M: int):
    """Bond sector tables for cuts 0..n with each bond capped at M states.

    Full sector dimensions are scaled down proportionally when they exceed M
    (every sector keeps at least one state).
    """
    bonds = []
    for c in range(n + 1):
        full = full_bond_sectors(n, n_alpha, n_beta, c)
        tot = sum(d for _, _, d in full)
        if tot <= M:
            bonds.append(full)
            continue
        scaled = [(N, s, max(1, int(d * M // tot))) for N, s, d in full]
        bonds.append(scaled)
    return bonds


def _index(bond):
    return {(N, s): i for i, (N, s, _) in enumerate(bond)}


def slab_shapes(bond_l, bond_r, phys_qn):
    """Per left sector: (m_l, [(phys index, right sector index, m_r)], width)."""
    ridx = _index(bond_r)
    shapes = []
    for (N, s2, ml) in bond_l:
        cols = []
        for p, (dN, ds) in enumerate(phys_qn):
            j = ridx.get((N + dN, s2 + ds))
            if j is not None:
                cols.append((p, j, bond_r[j][2]))
        shapes.append((ml, cols, sum(c[2] for c in cols)))
    return shapes


def twosite_qn():
    return [(SITE_QN[a][0] + SITE_QN[b][0], SITE_QN[a][1] + SITE_QN[b][1])
            for a in range(4) for b in range(4)]


def tensor_size(bond_l, bond_r, phys_qn):
    return sum(ml * w for ml, _, w in slab_shapes(bond_l, bond_r, phys_qn))


def random_mps(n: int, n_alpha: int, n_beta: int, M: int, seed: int = 1):
    """Random block-sparse MPS: dict(bonds=[...], sites=[flat float64 arrays])."""
    rng = np.random.default_rng(seed)
    bonds = bond_sectors(n, n_alpha, n_beta, M)
    sites = []
    for k in range(n):
        parts = []
        for ml, _, w in slab_shapes(bonds[k], bonds[k + 1], SITE_QN):
            # rows of roughly unit norm keep the state's scale O(1) along the chain
            parts.append(rng.normal(0.0, 1.0, ml * w) / np.sqrt(max(w, 1)))
        sites.append(np.concatenate(parts) if parts else np.zeros(0))
    return {"bonds": bonds, "sites": sites}


def random_twosite(bonds, k: int, seed: int = 2):
    """Random normalised two-site vector for sites (k, k+1) in slab layout."""
    rng = np.random.default_rng(seed)
    size = tensor_size(bonds[k], bonds[k + 2], twosite_qn())
    v = rng.normal(0.0, 1.0, size)
    return v / np.linalg.norm(v)
