"""Two-site truncation by per-sector SVD.  TEST INFRASTRUCTURE ONLY (see
``oracle/__init__.py``).

The decimation of the two-site step (Fig. 2 / Sec. II.H: keep chi_k states,
discard tau = the sum of the squared discarded singular values):

* psi[a s1 s2 b] is read as a matrix with rows (a, s1) and columns (s2, b);
  it is block diagonal in the middle-bond label q_m = q_a + q_s1 = q_b - q_s2,
  so the SVD splits into one SVD per middle sector.  Rows of a sector are
  ordered s1 = 0..3 (each left sector a = q_m - q_s1 of bond k), columns
  s2 = 0..3 (each right sector b = q_m + q_s2 of bond k+2).
* Several roots with weights w_r (state averaging): moving right (the kept
  side is the left, rows) the SVD is of the horizontal concatenation
  [sqrt(w_1) Psi_1 | sqrt(w_2) Psi_2 | ...]; moving left (kept side columns)
  of the vertical one.  Its singular values are the square roots of the
  eigenvalues of the weighted reduced density matrix.
* Singular values of all sectors are sorted together, descending.  When all
  of them fit in M nothing is dropped.  Otherwise the first M are kept, then
  values <= cut_rtol * s_1 are dropped from the end, then the cut moves up
  while it would split a cluster (s_keep - s_(keep+1) <= tie_rtol * s_1), so
  exactly degenerate values (e.g. mirror sectors (n_alpha, n_beta) and
  (n_beta, n_alpha) at S_z = 0) are kept or dropped together.  At least one
  value is kept.

The paper states only "keep chi_k, discard tau"; the sort, the cluster rule
and the thresholds are the readings listed with the design.

Pins (``tests/test_oracle_truncate.py``): a psi built from chosen sector
spectra U diag(s) V^T returns exactly those spectra, the chosen cut, tau and
the cluster rule on degenerate values straddling M; a single-sector psi
reduces to numpy's SVD of the plain matrix; the SA concatenation equals the
eigenvalues of the weighted density matrix.
"""
from __future__ import annotations

import numpy as np

from .blocks import SITE_QN, Bond, _add, _sub, twosite_qn, unpack


def middle_sectors(bond_k: Bond, bond_k2: Bond):
    """Middle labels q_m with their row parts [(s1, a)] and column parts [(s2, b)]."""
    mids = set()
    for a in range(len(bond_k)):
        for s1 in range(4):
            qm = _add(bond_k.q(a), SITE_QN[s1])
            for s2 in range(4):
                if bond_k2.find(_add(qm, SITE_QN[s2])) is not None:
                    mids.add(qm)
    out = []
    for qm in sorted(mids):
        rows = [(s1, bond_k.find(_sub(qm, SITE_QN[s1]))) for s1 in range(4)]
        rows = [(s1, a) for s1, a in rows if a is not None]
        cols = [(s2, bond_k2.find(_add(qm, SITE_QN[s2]))) for s2 in range(4)]
        cols = [(s2, b) for s2, b in cols if b is not None]
        out.append((qm, rows, cols))
    return out


def sector_matrix(blocks, bond_k, bond_k2, rows, cols):
    """Psi restricted to one middle sector, rows (s1, a), columns (s2, b)."""
    R = sum(bond_k.dim(a) for _, a in rows)
    C = sum(bond_k2.dim(b) for _, b in cols)
    M = np.zeros((R, C))
    r0 = 0
    for s1, a in rows:
        c0 = 0
        for s2, b in cols:
            blk = blocks.get((a, 4 * s1 + s2, b))
            if blk is not None:
                M[r0:r0 + bond_k.dim(a), c0:c0 + bond_k2.dim(b)] = blk
            c0 += bond_k2.dim(b)
        r0 += bond_k.dim(a)
    return M


def truncate(psis, bonds_k, bonds_k2, M, left_to_right=True, weights=None, tie_rtol=1e-10, cut_rtol=1e-14,
             trunc_tol=0.0, m_min=1):
    """Returns dict(bond=[(N, 2Sz, kept)] sorted, kept=descending kept values,
    tau, spectra={q_m: all singular values, descending}).

    trunc_tol > 0 (adaptive bond dimension): the first cut is the fewest values
    whose discarded weight sum(s^2) is at most trunc_tol times the total, raised
    to m_min; if that is below M it is taken and moved down the list (more kept)
    while it would split a cluster and M allows; the M rules above follow."""
    bk, bk2 = Bond(bonds_k), Bond(bonds_k2)
    psis = [np.asarray(p, dtype=float) for p in psis]
    nr = len(psis)
    w = np.full(nr, 1.0 / nr) if weights is None else np.asarray(weights, dtype=float) / np.sum(weights)
    blocks = [unpack(bk, bk2, twosite_qn(), p) for p in psis]
    spectra, allsv = {}, []
    for qm, rows, cols in middle_sectors(bk, bk2):
        mats = [np.sqrt(w[r]) * sector_matrix(blocks[r], bk, bk2, rows, cols) for r in range(nr)]
        big = np.hstack(mats) if left_to_right else np.vstack(mats)
        if big.size == 0:
            continue
        s = np.linalg.svd(big, compute_uv=False)
        spectra[qm] = s
        allsv.extend((v, qm) for v in s)
    allsv.sort(key=lambda t: -t[0])
    vals = np.array([v for v, _ in allsv])
    keep = min(len(vals), M)
    s1 = vals[0] if len(vals) else 0.0
    if trunc_tol > 0 and len(vals):
        total = float(np.sum(vals ** 2))
        kt = len(vals)
        while kt > 1 and float(np.sum(vals[kt - 1:] ** 2)) <= trunc_tol * total:
            kt -= 1
        kt = max(kt, m_min)
        if kt < keep:
            keep = kt
            while keep < min(len(vals), M) and vals[keep - 1] - vals[keep] <= tie_rtol * s1:
                keep += 1
    if keep < len(vals):
        while keep > 0 and vals[keep - 1] <= cut_rtol * s1:
            keep -= 1
        while keep > 1 and vals[keep - 1] - vals[keep] <= tie_rtol * s1:
            keep -= 1
    keep = max(keep, 1)
    tau = float(np.sum(vals[keep:] ** 2))
    count = {}
    for v, qm in allsv[:keep]:
        count[qm] = count.get(qm, 0) + 1
    bond = sorted((qm[0], qm[1], c) for qm, c in count.items())
    return {"bond": bond, "kept": vals[:keep].copy(), "tau": tau, "spectra": spectra}


def psi_from_spectra(bonds_k, bonds_k2, spectra, seed=0):
    """A two-site vector (slab layout) whose middle-sector singular values are
    the given ones: spectra = {q_m: values}; each sector gets seeded random
    orthonormal U, V (values beyond min(R, C) are ignored, sectors not listed
    are zero)."""
    from .blocks import pack
    bk, bk2 = Bond(bonds_k), Bond(bonds_k2)
    rng = np.random.default_rng(seed)
    blocks = {}
    for qm, rows, cols in middle_sectors(bk, bk2):
        if qm not in spectra:
            continue
        R = sum(bk.dim(a) for _, a in rows)
        C = sum(bk2.dim(b) for _, b in cols)
        s = np.asarray(spectra[qm], dtype=float)[:min(R, C)]
        if s.size == 0:
            continue
        U, _ = np.linalg.qr(rng.standard_normal((R, len(s))))
        V, _ = np.linalg.qr(rng.standard_normal((C, len(s))))
        Mq = (U * s) @ V.T
        r0 = 0
        for s1, a in rows:
            c0 = 0
            for s2, b in cols:
                blocks[(a, 4 * s1 + s2, b)] = Mq[r0:r0 + bk.dim(a), c0:c0 + bk2.dim(b)].copy()
                c0 += bk2.dim(b)
            r0 += bk.dim(a)
    return pack(bk, bk2, twosite_qn(), blocks)
