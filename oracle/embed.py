"""MPS -> determinant embedding and the two-site projected sigma.

An MPS is a plain tensor network over the site-product (interleaved
Jordan-Wigner) basis: spin orbitals ordered 0a, 0b, 1a, 1b, ..., site state
s = n_alpha + 2 n_beta, so |alpha beta> = a+_alpha a+_beta |0> on a site.
Reordering the creators of such a state into the determinant order (all alpha
first) passes each occupied alpha orbital p over the occupied beta orbitals
q < p, so

    c[I_a, I_b] = (-1)^(sum_p n_{p alpha} sum_{q<p} n_{q beta}) v[site-product index].

(The paper states no ordering or sign convention; this reading is pinned by
brute force in ``tests/test_oracle_embed.py``: the interleaved Fock-space H
equals S H_det S with S this sign.)

The two-site effective Hamiltonian of a DMRG step on sites (k, k+1) is the
projection of H onto span{|a> (x) |s1> (x) |s2> (x) |b>} where |a>, |b> are the
left/right block states the MPS defines (Fig. 2 of the paper: left block,
two sites, right block).  For a given MPS basis,

    sigma = P^T H P psi,   P psi = sum_{a s1 s2 b} psi[a s1 s2 b] |a s1 s2 b>,

computed here by building P explicitly from the MPS (dense, tiny n only) and
applying the determinant-space H of ``oracle.fci``.  This is the definition of
H_eff psi and needs no MPO or environment.
"""
from __future__ import annotations

import numpy as np

from . import fci

SITE_QN = ((0, 0), (1, 1), (1, -1), (2, 0))


def _offsets(bond):
    off, o = {}, 0
    for (N, s, d) in bond:
        off[(N, s)] = (o, d)
        o += d
    return off, o


def _slab_blocks(bond_l, bond_r, phys_qn):
    """Yield (left offset, m_l, phys, right offset, m_r, flat start, row stride, col start)."""
    offl, _ = _offsets(bond_l)
    offr, _ = _offsets(bond_r)
    flat = 0
    for (N, s2, ml) in bond_l:
        cols = []
        for p, (dN, ds) in enumerate(phys_qn):
            key = (N + dN, s2 + ds)
            if key in offr:
                cols.append((p, offr[key][0], offr[key][1]))
        width = sum(c[2] for c in cols)
        c0 = 0
        for (p, ro, mr) in cols:
            yield offl[(N, s2)][0], ml, p, ro, mr, flat, width, c0
            c0 += mr
        flat += ml * width


def slab_to_dense(bond_l, bond_r, phys_qn, flat):
    """Dense tensor [D_l, n_phys, D_r] from the slab storage (zeros elsewhere)."""
    _, Dl = _offsets(bond_l)
    _, Dr = _offsets(bond_r)
    T = np.zeros((Dl, len(phys_qn), Dr))
    for lo, ml, p, ro, mr, start, width, c0 in _slab_blocks(bond_l, bond_r, phys_qn):
        blk = flat[start:start + ml * width].reshape(ml, width)[:, c0:c0 + mr]
        T[lo:lo + ml, p, ro:ro + mr] = blk
    return T


def dense_to_slab(bond_l, bond_r, phys_qn, T):
    size = 0
    parts = {}
    for lo, ml, p, ro, mr, start, width, c0 in _slab_blocks(bond_l, bond_r, phys_qn):
        parts.setdefault(start, (ml, width, []))[2].append((c0, T[lo:lo + ml, p, ro:ro + mr]))
        size = max(size, start + ml * width)
    out = np.zeros(size)
    for start, (ml, width, blocks) in parts.items():
        slab = np.zeros((ml, width))
        for c0, b in blocks:
            slab[:, c0:c0 + b.shape[1]] = b
        out[start:start + ml * width] = slab.reshape(-1)
    return out


def twosite_qn():
    return [(SITE_QN[a][0] + SITE_QN[b][0], SITE_QN[a][1] + SITE_QN[b][1])
            for a in range(4) for b in range(4)]


def site_tensors(mps):
    bonds = mps["bonds"]
    return [slab_to_dense(bonds[k], bonds[k + 1], SITE_QN, mps["sites"][k])
            for k in range(len(mps["sites"]))]


def left_basis(A, k):
    """U[x, a]: left-block states at bond k as vectors over 4^k site-product states."""
    U = np.ones((1, 1))
    for j in range(k):
        U = np.einsum("xa,asb->xsb", U, A[j]).reshape(-1, A[j].shape[2])
    return U


def right_basis(A, k):
    """V[y, b]: right-block states at bond k (sites k..L-1) over 4^(L-k) states."""
    L = len(A)
    V = np.ones((1, 1))
    for j in range(L - 1, k - 1, -1):
        V = np.einsum("asb,yb->asy", A[j], V)
        V = V.reshape(A[j].shape[0], -1).T
    return V


def det_map(n, n_alpha, n_beta):
    """(site-product index, sign) of every determinant in FCI (colex) order."""
    sa = fci.strings(n, n_alpha)
    sb = fci.strings(n, n_beta)
    idx = np.zeros((len(sa), len(sb)), dtype=np.int64)
    sgn = np.ones((len(sa), len(sb)))
    for i, a in enumerate(sa):
        for j, b in enumerate(sb):
            x, parity, nb_below = 0, 0, 0
            for p in range(n):
                na_p = (int(a) >> p) & 1
                nb_p = (int(b) >> p) & 1
                x = 4 * x + na_p + 2 * nb_p
                parity += na_p * nb_below
                nb_below += nb_p
            idx[i, j] = x
            sgn[i, j] = -1.0 if parity & 1 else 1.0
    return idx, sgn


def fock_to_det(v, dm):
    idx, sgn = dm
    return sgn * v[idx]


def det_to_fock(c, dm, size):
    idx, sgn = dm
    v = np.zeros(size)
    v[idx] = sgn * c
    return v


def sigma_twosite(h, B, mps, k, psi_flat, n_alpha, n_beta, e_core=0.0):
    """Oracle H_eff psi for the two-site step on sites (k, k+1), slab layout in and out."""
    bonds = mps["bonds"]
    n = len(mps["sites"])
    A = site_tensors(mps)
    U = left_basis(A, k)
    V = right_basis(A, k + 2)
    psi = slab_to_dense(bonds[k], bonds[k + 2], twosite_qn(), psi_flat)
    psi = psi.reshape(psi.shape[0], 4, 4, psi.shape[2])
    full = np.einsum("xa,asub,yb->xsuy", U, psi, V).reshape(-1)
    dm = det_map(n, n_alpha, n_beta)
    space = fci.DetSpace(n, n_alpha, n_beta)
    c = fock_to_det(full, dm)
    leak = np.linalg.norm(full) ** 2 - np.linalg.norm(c) ** 2
    assert abs(leak) <= 1e-10 * max(1.0, np.linalg.norm(full) ** 2), "psi leaves the sector"
    s = fci.sigma(space, h, fci.eri(B), c, e_core)
    sf = det_to_fock(s, dm, full.size).reshape(U.shape[0], 4, 4, V.shape[0])
    out = np.einsum("xa,xsuy,yb->asub", U, sf, V)
    out = out.reshape(out.shape[0], 16, out.shape[3])
    return dense_to_slab(bonds[k], bonds[k + 2], twosite_qn(), out)


def mps_state(mps, n_alpha, n_beta):
    """Full CI vector c[I_a, I_b] of an MPS (tiny n)."""
    A = site_tensors(mps)
    n = len(A)
    full = left_basis(A, n).reshape(-1)
    return fock_to_det(full, det_map(n, n_alpha, n_beta))


def mps_energy(h, B, mps, n_alpha, n_beta, e_core=0.0):
    n = h.shape[0]
    c = mps_state(mps, n_alpha, n_beta)
    space = fci.DetSpace(n, n_alpha, n_beta)
    s = fci.sigma(space, h, fci.eri(B), c, e_core)
    return float(np.sum(c * s) / np.sum(c * c))


def project_twosite(mps, k, other):
    """Projection of the state `other` (an MPS of the same sites and sector) into
    the two-site space of `mps` at step k (sites k, k+1), slab layout:
    phi[a s1 s2 b] = sum_{x, y} U[x, a] Phi[x s1 s2 y] V[y, b], with U, V the
    left / right block states of `mps` over the site-product basis (Sec. II.F:
    a lower state seen from the two-site optimisation of another)."""
    bonds = mps["bonds"]
    A = site_tensors(mps)
    U = left_basis(A, k)
    V = right_basis(A, k + 2)
    F = site_tensors(other)
    full = left_basis(F, len(F)).reshape(-1)
    full = full.reshape(U.shape[0], 4, 4, V.shape[0])
    out = np.einsum("xa,xsuy,yb->asub", U, full, V)
    out = out.reshape(out.shape[0], 16, out.shape[3])
    return dense_to_slab(bonds[k], bonds[k + 2], twosite_qn(), out)


def overlap(mps_a, mps_b):
    """<A|B> / (||A|| ||B||) of two MPS over the site-product basis."""
    a = left_basis(site_tensors(mps_a), len(mps_a["sites"])).reshape(-1)
    b = left_basis(site_tensors(mps_b), len(mps_b["sites"])).reshape(-1)
    return float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))
