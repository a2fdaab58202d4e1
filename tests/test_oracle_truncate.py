"""Pins of the oracle truncation (oracle.truncate): chosen sector spectra come
back exactly, the cut with the cluster rule, tau, single-sector SVD and the
state-averaged density-matrix identity."""
import numpy as np

import synth
from oracle import blocks, truncate

N, NA, NB, M, K = 6, 3, 3, 20, 2


def _bonds():
    mps = synth.random_mps(N, NA, NB, M, seed=4)
    return mps["bonds"][K], mps["bonds"][K + 2]


def test_spectra_roundtrip_and_cut():
    bk, bk2 = _bonds()
    mids = truncate.middle_sectors(blocks.Bond(bk), blocks.Bond(bk2))
    rng = np.random.default_rng(0)
    spectra = {}
    for qm, rows, cols in mids:
        R = sum(blocks.Bond(bk).dim(a) for _, a in rows)
        C = sum(blocks.Bond(bk2).dim(b) for _, b in cols)
        spectra[qm] = np.sort(rng.uniform(0.01, 1.0, min(R, C)))[::-1]
    psi = truncate.psi_from_spectra(bk, bk2, spectra, seed=1)
    res = truncate.truncate([psi], bk, bk2, M=10 ** 6)
    for qm, s in spectra.items():
        assert np.allclose(res["spectra"][qm], s, atol=1e-13)
    allv = np.sort(np.concatenate(list(spectra.values())))[::-1]
    assert res["tau"] == 0.0 and len(res["kept"]) == len(allv)
    # a cut of 7 keeps the 7 largest, tau is the rest (all values distinct here)
    res7 = truncate.truncate([psi], bk, bk2, M=7)
    assert np.allclose(res7["kept"], allv[:7], atol=1e-13)
    assert abs(res7["tau"] - np.sum(allv[7:] ** 2)) < 1e-12
    assert sum(c for _, _, c in res7["bond"]) == 7


def test_cluster_rule_keeps_degenerate_values_together():
    """Mirror sectors (N, +2Sz) and (N, -2Sz) with equal values straddling the cut."""
    bk, bk2 = _bonds()
    bK, bK2 = blocks.Bond(bk), blocks.Bond(bk2)
    size = {}
    for qm, rows, cols in truncate.middle_sectors(bK, bK2):
        size[qm] = min(sum(bK.dim(a) for _, a in rows), sum(bK2.dim(b) for _, b in cols))
    pair = next(q for q in size if q[1] > 0 and size[q] >= 2 and size.get((q[0], -q[1]), 0) >= 2)
    mirror = (pair[0], -pair[1])
    big = next(q for q in size if q not in (pair, mirror) and size[q] >= 3)
    spectra = {big: [0.9, 0.5, 0.3], pair: [0.7, 0.2], mirror: [0.7, 0.2]}
    psi = truncate.psi_from_spectra(bk, bk2, spectra, seed=3)
    vals = np.sort(np.concatenate([np.asarray(v, float) for v in spectra.values()]))[::-1]
    # M between the two copies of 0.2: the cut moves up to keep neither
    first02 = int(np.nonzero(np.isclose(vals, 0.2))[0][0])
    res = truncate.truncate([psi], bk, bk2, M=first02 + 1)
    kept = res["kept"]
    assert not np.any(np.isclose(kept, 0.2)), "a degenerate cluster was split"
    assert len(kept) == first02
    assert abs(res["tau"] - np.sum(vals[first02:] ** 2)) < 1e-12
    # the degenerate values are exact here: the rule sees them as one cluster
    assert abs(res["spectra"][pair][1] - res["spectra"][mirror][1]) < 1e-14
    # one more state keeps both copies
    res2 = truncate.truncate([psi], bk, bk2, M=first02 + 2)
    assert np.sum(np.isclose(res2["kept"], 0.2)) == 2
    assert abs(res2["tau"]) < 1e-24


def test_cut_rtol_drops_tiny_values_only_when_truncating():
    bk, bk2 = _bonds()
    qms = [qm for qm, _, _ in truncate.middle_sectors(blocks.Bond(bk), blocks.Bond(bk2))]
    spectra = {qms[0]: [1.0, 1e-16], qms[1]: [0.5]}
    psi = truncate.psi_from_spectra(bk, bk2, spectra, seed=5)
    full = truncate.truncate([psi], bk, bk2, M=100, cut_rtol=1e-14)
    assert len(full["kept"]) >= 3  # everything fits: nothing dropped (zeros included)
    cut = truncate.truncate([psi], bk, bk2, M=2, cut_rtol=1e-14)
    assert len(cut["kept"]) == 2 and np.allclose(cut["kept"], [1.0, 0.5])


def test_single_sector_is_numpy_svd_and_sa_is_density_matrix():
    bk, bk2 = _bonds()
    bK, bK2 = blocks.Bond(bk), blocks.Bond(bk2)
    psi1 = synth.random_twosite([None] * K + [bk, None, bk2], K, seed=7)
    psi2 = synth.random_twosite([None] * K + [bk, None, bk2], K, seed=8)
    res = truncate.truncate([psi1], bk, bk2, M=10 ** 6)
    b1 = blocks.unpack(bK, bK2, blocks.twosite_qn(), psi1)
    b2 = blocks.unpack(bK, bK2, blocks.twosite_qn(), psi2)
    w = np.array([0.3, 0.7])
    sa_r = truncate.truncate([psi1, psi2], bk, bk2, M=10 ** 6, weights=w, left_to_right=True)
    sa_l = truncate.truncate([psi1, psi2], bk, bk2, M=10 ** 6, weights=w, left_to_right=False)
    for qm, rows, cols in truncate.middle_sectors(bK, bK2):
        P1 = truncate.sector_matrix(b1, bK, bK2, rows, cols)
        P2 = truncate.sector_matrix(b2, bK, bK2, rows, cols)
        assert np.allclose(res["spectra"][qm], np.linalg.svd(P1, compute_uv=False), atol=1e-13)
        rho = w[0] * P1 @ P1.T + w[1] * P2 @ P2.T
        ev = np.sort(np.clip(np.linalg.eigvalsh(rho), 0, None))[::-1]
        n = len(sa_r["spectra"][qm])
        assert np.allclose(sa_r["spectra"][qm] ** 2, ev[:n], atol=1e-13)
        rho_c = w[0] * P1.T @ P1 + w[1] * P2.T @ P2
        evc = np.sort(np.clip(np.linalg.eigvalsh(rho_c), 0, None))[::-1]
        n = len(sa_l["spectra"][qm])
        assert np.allclose(sa_l["spectra"][qm] ** 2, evc[:n], atol=1e-13)


def _pair_spectra():
    """A big sector [0.9, 0.5, 0.3] and a mirror pair of sectors with [0.7, 0.2]
    each, normalised; returns (bk, bk2, psi, sorted values, index of the first 0.2)."""
    bk, bk2 = _bonds()
    bK, bK2 = blocks.Bond(bk), blocks.Bond(bk2)
    size = {}
    for qm, rows, cols in truncate.middle_sectors(bK, bK2):
        size[qm] = min(sum(bK.dim(a) for _, a in rows), sum(bK2.dim(b) for _, b in cols))
    pair = next(q for q in size if q[1] > 0 and size[q] >= 2 and size.get((q[0], -q[1]), 0) >= 2)
    big = next(q for q in size if q not in (pair, (pair[0], -pair[1])) and size[q] >= 3)
    spectra = {big: [0.9, 0.5, 0.3], pair: [0.7, 0.2], (pair[0], -pair[1]): [0.7, 0.2]}
    tot = np.sqrt(sum(np.sum(np.square(v)) for v in spectra.values()))
    spectra = {q: np.asarray(v) / tot for q, v in spectra.items()}
    psi = truncate.psi_from_spectra(bk, bk2, spectra, seed=3)
    vals = np.sort(np.concatenate(list(spectra.values())))[::-1]
    return bk, bk2, psi, vals, int(np.nonzero(np.isclose(vals, 0.2 / tot))[0][0])


def test_adaptive_cut_is_the_fewest_states_within_the_tolerance():
    bk, bk2, psi, vals, _ = _pair_spectra()  # 0.9, 0.7, 0.7, 0.5, 0.3, 0.2, 0.2 (scaled)
    w = vals ** 2
    # tolerance between the weights of the last value and of the last three:
    # dropping 0.3 and both 0.2 stays within it, dropping 0.5 too does not
    tol = 0.5 * (np.sum(w[4:]) + np.sum(w[3:]))
    res = truncate.truncate([psi], bk, bk2, M=100, trunc_tol=tol)
    assert len(res["kept"]) == 4 and res["tau"] <= tol and abs(res["tau"] - np.sum(w[4:])) < 1e-13
    # M still caps the count; m_min raises it
    assert len(truncate.truncate([psi], bk, bk2, M=3, trunc_tol=tol)["kept"]) == 3
    assert len(truncate.truncate([psi], bk, bk2, M=100, trunc_tol=tol, m_min=6)["kept"]) == 7  # cluster kept whole
    assert len(truncate.truncate([psi], bk, bk2, M=100, trunc_tol=0.99)["kept"]) == 1
    # trunc_tol = 0 is the fixed-M rule: everything fits, nothing goes (zeros included)
    assert len(truncate.truncate([psi], bk, bk2, M=100, trunc_tol=0.0)["kept"]) > 7


def test_adaptive_cut_keeps_a_cluster_whole():
    """The tolerance would keep one copy of the degenerate pair: the cut moves
    down the list to keep both while M allows, else the M rule drops both."""
    bk, bk2, psi, vals, first02 = _pair_spectra()
    w = vals ** 2
    tol = 0.5 * (w[-1] + np.sum(w[-2:]))  # allows dropping one copy only
    res = truncate.truncate([psi], bk, bk2, M=100, trunc_tol=tol)
    assert len(res["kept"]) == first02 + 2 and res["tau"] < 1e-24
    capped = truncate.truncate([psi], bk, bk2, M=first02 + 1, trunc_tol=tol)
    assert len(capped["kept"]) == first02
