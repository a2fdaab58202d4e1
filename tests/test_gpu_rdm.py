"""Determinant-space view and (transition) 1-/2-RDMs on the GPU, through the C
ABI, against the CPU oracle: the CI vector of an MPS (ragged truncated bonds,
odd chains, empty spin strings, held states), transition RDMs of random CI
vectors element-wise, multi-pass RDMs at CAS(12,11) on sampled elements and the
energy identity, and the RDMs of converged DMRG roots against FCI."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import embed, fci

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fci_energies.json")


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("n,na,nb,M,seed", [
    (2, 1, 0, 4, 1),      # two sites, no beta electrons (one empty beta string)
    (4, 2, 2, 16, 1),     # full bonds
    (5, 3, 2, 8, 2),      # odd chain, truncated
    (6, 3, 3, 12, 5),     # ragged sectors
    (6, 0, 3, 10, 3),     # no alpha electrons: one (empty) alpha string
    (7, 4, 2, 20, 7),
    (8, 4, 4, 40, 9),
    (10, 5, 5, 200, 4),
])
def test_mps_to_ci_matches_oracle(n, na, nb, M, seed):
    torch = _torch()
    import paper_2609_09990_amd as pk
    print(f"mps_to_ci n={n} ({na},{nb}) M={M}", flush=True)
    h, B, e0 = synth.make_hamiltonian(n, 4, 0)
    mps = synth.random_mps(n, na, nb, M, seed=seed)
    sol = pk.Solver(pk.Problem(h, B, na, nb, e0), M=M)
    sol.set_mps(mps["bonds"], mps["sites"])
    got = sol.mps_to_ci().cpu().numpy()
    ref = embed.mps_state(mps, na, nb)
    assert got.shape == ref.shape
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    # a held state
    other = synth.random_mps(n, na, nb, max(2, M // 2), seed=seed + 1)
    sol.deflate(other, 1.0)
    got1 = sol.mps_to_ci(1).cpu().numpy()
    ref1 = embed.mps_state(other, na, nb)
    assert np.abs(got1 - ref1).max() <= 1e-13 * np.abs(ref1).max()


@pytest.mark.parametrize("n,na,nb,same", [(2, 1, 1, False), (4, 2, 2, False), (5, 3, 1, False), (6, 3, 3, False),
                                          (6, 3, 3, True), (7, 4, 3, False), (8, 4, 4, True)])
def test_ci_rdm12_matches_oracle(n, na, nb, same):
    """Random CI vectors: every element of gamma and Gamma' against the oracle's
    nested application of E (relative to the largest element, 1e-12)."""
    torch = _torch()
    import paper_2609_09990_amd as pk
    print(f"ci_rdm12 n={n} ({na},{nb}) same={same}", flush=True)
    h, B, e0 = synth.make_hamiltonian(n, 4, 0)
    prob = pk.Problem(h, B, na, nb, e0)
    space = fci.DetSpace(n, na, nb)
    rng = np.random.default_rng(n * 7 + na)
    bra = rng.normal(size=space.shape)
    ket = bra if same else rng.normal(size=space.shape)
    db = torch.from_numpy(bra).cuda()
    dk = db if same else torch.from_numpy(ket).cuda()
    g, G, ov = prob.ci_rdm12(db, dk)
    rg, rG = fci.trdm12(space, bra, ket)
    scale = max(np.abs(rG).max(), 1.0)
    assert np.abs(g - rg).max() <= 1e-12 * scale
    assert np.abs(G - rG).max() <= 1e-12 * scale
    assert abs(ov - float(np.sum(bra * ket))) <= 1e-12 * np.sum(bra * bra) ** 0.5 * np.sum(ket * ket) ** 0.5


def test_multipass_rdm12_cas12_sampled_and_energy():
    """CAS(12,11) (6 alpha, 5 beta, 731,808 determinants: two passes of excited
    copies): gamma element-wise, 40 sampled Gamma' elements one by one, and
    E = h.gamma + 1/2 (pq|rs) Gamma' equal to the oracle's <c|H|c> / <c|c>."""
    torch = _torch()
    import paper_2609_09990_amd as pk
    n, na, nb = 12, 6, 5
    h, B, e0 = synth.make_hamiltonian(n, 24, 3)
    prob = pk.Problem(h, B, na, nb, e0)
    space = fci.DetSpace(n, na, nb)
    rng = np.random.default_rng(12)
    c = rng.normal(size=space.shape)
    g, G, ov = prob.ci_rdm12(torch.from_numpy(c).cuda())
    rg = np.array([[np.sum(c * space.apply_E(p, q, c)) for q in range(n)] for p in range(n)])
    assert np.abs(g - rg).max() <= 1e-12 * np.abs(rg).max()
    for _ in range(40):
        p, q, r, s = (int(x) for x in rng.integers(0, n, size=4))
        ref = np.sum(space.apply_E(q, p, c) * space.apply_E(r, s, c)) - (q == r) * rg[p, s]
        assert abs(G[p, q, r, s] - ref) <= 1e-12 * np.abs(rg).max(), (p, q, r, s)
    e = fci.energy_from_rdm(h, B, g, G, e0) / ov
    ref_e = float(np.sum(c * fci.sigma(space, h, fci.eri(B), c, e0))) / float(np.sum(c * c))
    print(f"E(RDM) {e:.12f} vs <H> {ref_e:.12f}", flush=True)
    assert abs(e - ref_e) <= 1e-11 * abs(ref_e)


def test_rdms_of_dmrg_roots_equal_fci():
    """CAS(8,8), N_Q = 32 at full bond: the 1-/2-RDMs of the DMRG ground state
    and the transition RDMs between it and the first excited root (penalty
    deflation) equal those of the oracle's FCI vectors (up to each root's sign);
    <1|H|0> from the transition RDMs vanishes."""
    _torch()
    import paper_2609_09990_amd as pk
    g = json.load(open(GOLD))["cas8_nq32_s0"]
    h, B, e0 = synth.make_hamiltonian(8, 32, 0)
    prob = pk.Problem(h, B, 4, 4, e0)
    res = pk.excited_states(prob, 2, M=256, tol=1e-10, sweeps=3, conv_tol=1e-11)
    assert np.max(np.abs(res["energies"] - np.array(g["energies"][:2]))) <= 1e-10
    w, vs, space = fci.solve(8, 4, 4, h, B, nroots=2, e_core=e0, tol=1e-12)
    sol = pk.Solver(prob, M=256)
    m1 = res["mps"][1]
    sol.set_mps(m1["bonds"], m1["sites"])
    sol.deflate(res["mps"][0], 1.0)
    g00, G00, o00 = sol.rdm12(1, 1)
    r00, R00 = fci.rdm12(space, vs[0])
    assert abs(o00 - 1.0) <= 1e-12
    assert np.abs(g00 - r00).max() <= 1e-8 and np.abs(G00 - R00).max() <= 1e-8
    g10, G10, o10 = sol.rdm12(0, 1)
    r10, R10 = fci.trdm12(space, vs[1], vs[0])
    sgn = 1.0 if np.sum(g10 * r10) >= 0 else -1.0
    print(f"|<1|0>| {abs(o10):.1e}, transition gamma err {np.abs(g10 - sgn * r10).max():.1e}", flush=True)
    assert abs(o10) <= 1e-6
    assert np.abs(g10 - sgn * r10).max() <= 1e-7 and np.abs(G10 - sgn * R10).max() <= 1e-7
    assert abs(fci.energy_from_rdm(h, B, g10, G10)) <= 1e-8
    assert abs(fci.energy_from_rdm(h, B, g00, G00, e0) - res["energies"][0]) <= 1e-9


def _v_ref(space, B, c):
    g = fci.eri(B)
    return fci.sigma(space, 0.5 * np.einsum("prrq->pq", g), g, c)


@pytest.mark.parametrize("n,na,nb,nq", [(4, 2, 2, 5), (6, 3, 3, 8), (8, 4, 4, 32), (10, 5, 4, 12)])
def test_ci_apply_v_matches_oracle(n, na, nb, nq):
    """V c (the two-electron block streamed through the Cholesky factors)
    against the oracle's Hamiltonian action without its one-body part."""
    torch = _torch()
    import paper_2609_09990_amd as pk
    print(f"apply_v n={n} ({na},{nb}) nq={nq}", flush=True)
    h, B, e0 = synth.make_hamiltonian(n, nq, 1)
    prob = pk.Problem(h, B, na, nb, e0)
    space = fci.DetSpace(n, na, nb)
    c = np.random.default_rng(n).normal(size=space.shape)
    got = prob.ci_apply_v(torch.from_numpy(c).cuda()).cpu().numpy()
    ref = _v_ref(space, B, c)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("n,na,nb,full", [(3, 2, 1, True), (4, 2, 2, True), (5, 3, 2, True), (8, 4, 4, False),
                                          (10, 5, 5, False)])
def test_ci_rdm3_matches_oracle(n, na, nb, full):
    """<bra|E_pq E_rs E_tu|ket>: every element (n <= 5) or 60 sampled elements
    and the trace identity sum_t Gamma3[pqrstt] = N <bra|E_pq E_rs|ket> (n = 8,
    and n = 10 where the determinants take two passes)."""
    torch = _torch()
    import paper_2609_09990_amd as pk
    print(f"rdm3 n={n} ({na},{nb})", flush=True)
    h, B, e0 = synth.make_hamiltonian(n, 4, 0)
    prob = pk.Problem(h, B, na, nb, e0)
    space = fci.DetSpace(n, na, nb)
    rng = np.random.default_rng(3 * n)
    bra, ket = rng.normal(size=(2,) + space.shape)
    db, dk = torch.from_numpy(bra).cuda(), torch.from_numpy(ket).cuda()
    G3 = prob.ci_rdm3(db, dk)
    if full:
        ref = fci.rdm3(space, bra, ket)
        assert np.abs(G3 - ref).max() <= 1e-12 * np.abs(ref).max()
        return
    picks = [tuple(int(x) for x in rng.integers(0, n, size=6)) for _ in range(60)]
    ref = fci.rdm3(space, bra, ket, picks)
    scale = np.abs(G3).max()
    for x, r in zip(picks, ref):
        assert abs(G3[x] - r) <= 1e-12 * scale, x
    g, G, _ = prob.ci_rdm12(db, dk)
    EE = G + np.einsum("qr,ps->pqrs", np.eye(n), g)
    assert np.abs(np.einsum("pqrstt->pqrs", G3) - (na + nb) * EE).max() <= 1e-11 * scale


def test_fused_four_body_contraction_cas8():
    """CAS(8,8), N_Q = 32, the DMRG ground state's CI vector c: the
    four-particle density contracted with the two-electron block,
    sum_vwxy (vw|xy)/2 <c|E_pq E_rs E_tu E_vw E_xy|c>, as the three-body density
    of (c, V c) (the n^8 object never formed), against the oracle on 40 sampled
    elements; and its full contraction with delta_pq delta_rs delta_tu equals
    N^3 <c|V|c>."""
    torch = _torch()
    import paper_2609_09990_amd as pk
    h, B, e0 = synth.make_hamiltonian(8, 32, 0)
    prob = pk.Problem(h, B, 4, 4, e0)
    sol = pk.Solver(prob, M=256, tol=1e-10)
    sol.sweep(3)
    c = sol.mps_to_ci()
    vc = prob.ci_apply_v(c)
    F = prob.ci_rdm3(c, vc)
    space = fci.DetSpace(8, 4, 4)
    ch = c.cpu().numpy()
    vref = _v_ref(space, B, ch)
    rng = np.random.default_rng(8)
    picks = [tuple(int(x) for x in rng.integers(0, 8, size=6)) for _ in range(40)]
    ref = fci.rdm3(space, ch, vref, picks)
    scale = np.abs(F).max()
    for x, r in zip(picks, ref):
        assert abs(F[x] - r) <= 1e-11 * scale, x
    assert abs(np.einsum("pprrtt->", F) - 8 ** 3 * float(np.sum(ch * vref))) <= 1e-10 * abs(8 ** 3 * np.sum(ch * vref))


def test_mps_rdm1_from_the_gradient_at_any_size():
    """gamma = dE/dh (dmrg_grad) is the 1-RDM of the MPS at any size: equal to
    the CI route at CAS(10,10) after two sweeps at M = 64, and at CAS(16,16)
    M = 128 (no CI vector) symmetric with trace N and natural occupations in
    [0, 2]."""
    _torch()
    import paper_2609_09990_amd as pk
    h, B, e0 = synth.make_hamiltonian(10, 16, 2)
    prob = pk.Problem(h, B, 5, 5, e0)
    sol = pk.Solver(prob, M=64, tol=1e-8)
    sol.sweep(2)
    g_mps = sol.rdm1()
    g_ci, _, _ = sol.rdm12()
    assert np.abs(g_mps - g_ci).max() <= 1e-11
    h, B, e0 = synth.make_hamiltonian(16, 32, 1)
    sol = pk.Solver(pk.Problem(h, B, 8, 8, e0), M=128, tol=1e-7)
    sol.sweep(2)
    g = sol.rdm1()
    w = np.linalg.eigvalsh(0.5 * (g + g.T))
    print(f"CAS(16,16) natural occupations {w.min():.4f} .. {w.max():.4f}", flush=True)
    assert np.abs(g - g.T).max() <= 1e-10 and abs(np.trace(g) - 16) <= 1e-9
    assert w.min() >= -1e-10 and w.max() <= 2 + 1e-10
