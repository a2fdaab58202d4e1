"""Brute-force Jordan-Wigner Fock-space Hamiltonian (tiny n only).

States are bitmasks over spin-orbital *labels*: label(p, alpha) = p and
label(p, beta) = n + p.  The Jordan-Wigner order is a separate permutation
``pos[label]``: a ladder operator on label j acting on a state picks up the sign
(-1)^(number of occupied labels whose position is below pos[j]).  With the
alpha-first order (pos = identity) a state bitmask *is* the determinant
|I_a I_b> of the FCI module with sign +1; with the interleaved order
(0a, 0b, 1a, 1b, ...) it is the site-product basis an MPS is written in.

H = sum_pq h_pq sum_s a+_{p s} a_{q s}
  + 1/2 sum_pqru (pq|ru) sum_{s,t} a+_{p s} a+_{r t} a_{u t} a_{q s}
(normal ordered), applied term by term.

This is the textbook second-quantised Hamiltonian with no factorisation, no
string algebra and no Knowles-Handy reorganisation: it pins ``fci``.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def alpha_first_positions(n: int) -> np.ndarray:
    return np.arange(2 * n)


def interleaved_positions(n: int) -> np.ndarray:
    pos = np.empty(2 * n, dtype=np.int64)
    for p in range(n):
        pos[p] = 2 * p          # alpha
        pos[n + p] = 2 * p + 1  # beta
    return pos


def _below_masks(pos: np.ndarray) -> np.ndarray:
    """mask[j] = bitmask of labels whose JW position is below pos[j]."""
    m = np.zeros(len(pos), dtype=np.int64)
    for j in range(len(pos)):
        for i in range(len(pos)):
            if pos[i] < pos[j]:
                m[j] |= 1 << i
    return m


def _ladder(states, signs, j, create, below):
    occ = (states >> j) & 1
    ok = occ == (0 if create else 1)
    parity = np.zeros_like(states)
    x = states & below[j]
    while np.any(x):
        parity ^= x & 1
        x >>= 1
    new_signs = np.where(ok, signs * (1 - 2 * parity), 0)
    return states ^ (1 << j), new_signs


def hamiltonian(h, B, basis, pos, e_core=0.0):
    """Sparse H on the given list of bitmask states (the list must be closed
    under H, e.g. a fixed (N_alpha, N_beta) sector or the full Fock space)."""
    n = h.shape[0]
    g = np.einsum("Qpq,Qrs->pqrs", B, B)
    below = _below_masks(pos)
    basis = np.asarray(basis, dtype=np.int64)
    index = {int(s): i for i, s in enumerate(basis)}
    N = len(basis)
    rows, cols, vals = [list(range(N))], [list(range(N))], [[e_core] * N]

    def add_term(coef, ops):
        if coef == 0.0:
            return
        st = basis.copy()
        sg = np.ones(N, dtype=np.int64)
        for j, create in reversed(ops):  # rightmost operator acts first
            st, sg = _ladder(st, sg, j, create, below)
        nz = np.nonzero(sg)[0]
        if nz.size == 0:
            return
        rows.append([index[int(s)] for s in st[nz]])
        cols.append(list(nz))
        vals.append(list(coef * sg[nz]))

    for p in range(n):
        for q in range(n):
            for s in range(2):
                add_term(h[p, q], [(p + n * s, True), (q + n * s, False)])
    for p in range(n):
        for q in range(n):
            for r in range(n):
                for t in range(n):
                    c = 0.5 * g[p, q, r, t]
                    if abs(c) < 1e-300:
                        continue
                    for s1 in range(2):
                        for s2 in range(2):
                            add_term(c, [(p + n * s1, True), (r + n * s2, True),
                                         (t + n * s2, False), (q + n * s1, False)])
    r = np.concatenate([np.asarray(x, dtype=np.int64) for x in rows])
    c = np.concatenate([np.asarray(x, dtype=np.int64) for x in cols])
    v = np.concatenate([np.asarray(x, dtype=float) for x in vals])
    return sp.csr_matrix((v, (r, c)), shape=(N, N))


def sector_basis(n, n_alpha, n_beta):
    """Bitmask states with the given alpha / beta counts (labels as above)."""
    out = []
    for s in range(1 << (2 * n)):
        if bin(s & ((1 << n) - 1)).count("1") == n_alpha and bin(s >> n).count("1") == n_beta:
            out.append(s)
    return np.array(out, dtype=np.int64)


def site_product_basis(n):
    """Full Fock space in site-product order: index = sum_p s_p 4^(n-1-p),
    s_p = n_{p alpha} + 2 n_{p beta}; returns the label bitmask of each index."""
    out = np.zeros(4 ** n, dtype=np.int64)
    for idx in range(4 ** n):
        bits, x = 0, idx
        for p in range(n - 1, -1, -1):
            s = x % 4
            x //= 4
            if s & 1:
                bits |= 1 << p
            if s & 2:
                bits |= 1 << (n + p)
        out[idx] = bits
    return out
