"""Pins of the oracle's transition 1-/2-RDMs (fci.trdm12): products of
brute-force Fock-space one-body operators, a hand-worked two-orbital case,
the adjoint formulation of rdm12, traces, symmetries, and Hamiltonian matrix
elements between eigenstates.  CPU only."""
import numpy as np
import pytest

import synth
from oracle import fci, fock


def _fock_one_body(n, na, nb, p, q):
    """E_pq on the (na, nb) sector of the alpha-first Fock basis (= determinants)."""
    h = np.zeros((n, n))
    h[p, q] = 1.0
    basis = fock.sector_basis(n, na, nb)
    return fock.hamiltonian(h, np.zeros((0, n, n)), basis, fock.alpha_first_positions(n)), basis


def _to_fock(space, C, basis):
    n = space.n
    ia = {int(s): i for i, s in enumerate(space.sa)}
    ib = {int(s): i for i, s in enumerate(space.sb)}
    mask = (1 << n) - 1
    return np.array([C[ia[int(s) & mask], ib[int(s) >> n]] for s in basis])


@pytest.mark.parametrize("n,na,nb", [(3, 2, 1), (4, 2, 2), (4, 1, 3), (3, 0, 2)])
def test_trdm12_equals_fock_space_operator_products(n, na, nb):
    space = fci.DetSpace(n, na, nb)
    rng = np.random.default_rng(10 * n + na)
    bra, ket = rng.normal(size=(2,) + space.shape)
    g, G = fci.trdm12(space, bra, ket)
    E, basis = {}, None
    for p in range(n):
        for q in range(n):
            E[p, q], basis = _fock_one_body(n, na, nb, p, q)
    fb, fk = _to_fock(space, bra, basis), _to_fock(space, ket, basis)
    for p in range(n):
        for q in range(n):
            assert abs(g[p, q] - fb @ (E[p, q] @ fk)) < 1e-12
            for r in range(n):
                for s in range(n):
                    ref = fb @ (E[p, q] @ (E[r, s] @ fk)) - (q == r) * (fb @ (E[p, s] @ fk))
                    assert abs(G[p, q, r, s] - ref) < 1e-12, (p, q, r, s)


def test_trdm12_hand_example():
    """Two orbitals, one alpha and one beta electron: gamma_01 = <bra|E_01|ket>
    moves an electron from orbital 1 to 0 in the ket, alpha then beta, with no
    sign (nothing of the same spin lies between)."""
    space = fci.DetSpace(2, 1, 1)  # strings {0} (rank 0), {1} (rank 1)
    ket = np.array([[1.0, 2.0], [3.0, 4.0]])
    bra = np.array([[0.5, -1.0], [2.0, 0.25]])
    g, _ = fci.trdm12(space, bra, ket)
    # alpha: bra[0, b] ket[1, b]; beta: bra[a, 0] ket[a, 1]
    assert abs(g[0, 1] - ((0.5 * 3 - 1.0 * 4) + (0.5 * 2 + 2.0 * 4))) < 1e-14
    assert abs(g[1, 0] - ((2.0 * 1 + 0.25 * 2) + (-1.0 * 1 + 0.25 * 3))) < 1e-14
    assert abs(g[0, 0] - ((0.5 * 1 - 1.0 * 2) + (0.5 * 1 + 2.0 * 3))) < 1e-14


def test_trdm12_of_one_state_is_rdm12_and_properties():
    n, na, nb = 4, 2, 1
    space = fci.DetSpace(n, na, nb)
    rng = np.random.default_rng(3)
    a, b = rng.normal(size=(2,) + space.shape)
    g, G = fci.trdm12(space, a, a)
    g0, G0 = fci.rdm12(space, a)  # the adjoint formulation <E_qp a | E_rs a>
    assert np.abs(g - g0).max() < 1e-12 and np.abs(G - G0).max() < 1e-12
    gab, Gab = fci.trdm12(space, a, b)
    gba, Gba = fci.trdm12(space, b, a)
    N, ov = na + nb, float(np.sum(a * b))
    assert abs(np.trace(gab) - N * ov) < 1e-12
    assert np.abs(np.einsum("pqrr->pq", Gab) - (N - 1) * gab).max() < 1e-12
    assert np.abs(gab - gba.T).max() < 1e-12
    assert np.abs(Gab - Gba.transpose(1, 0, 3, 2)).max() < 1e-12
    assert np.abs(Gab - Gab.transpose(2, 3, 0, 1)).max() < 1e-12


def test_transition_rdms_give_hamiltonian_matrix_elements():
    n, na, nb = 4, 2, 2
    h, B, e0 = synth.make_hamiltonian(n, 6, 1)
    w, vs, space = fci.solve(n, na, nb, h, B, nroots=3, e_core=e0, tol=1e-12)
    for i in range(3):
        for j in range(3):
            g, G = fci.trdm12(space, vs[i], vs[j])
            e = fci.energy_from_rdm(h, B, g, G) + (e0 if i == j else 0.0)
            assert abs(e - (w[i] if i == j else 0.0)) < 1e-9, (i, j, e)


def test_apply_v_equals_sigma_without_one_body_part():
    """V = 1/2 sum (pq|rs) E_pq E_rs is the Hamiltonian of fci.sigma with
    h = 1/2 sum_r (pr|rq) (its one-body shift then cancels)."""
    n, na, nb = 4, 2, 1
    h, B, _ = synth.make_hamiltonian(n, 5, 7)
    space = fci.DetSpace(n, na, nb)
    C = np.random.default_rng(1).normal(size=space.shape)
    g = fci.eri(B)
    ref = fci.sigma(space, 0.5 * np.einsum("prrq->pq", g), g, C)
    assert np.abs(fci.apply_v(space, B, C) - ref).max() < 1e-12


@pytest.mark.parametrize("n,na,nb", [(3, 2, 1), (3, 1, 1)])
def test_rdm3_equals_fock_space_operator_products(n, na, nb):
    space = fci.DetSpace(n, na, nb)
    rng = np.random.default_rng(20 + n + na)
    bra, ket = rng.normal(size=(2,) + space.shape)
    G3 = fci.rdm3(space, bra, ket)
    E, basis = {}, None
    for p in range(n):
        for q in range(n):
            E[p, q], basis = _fock_one_body(n, na, nb, p, q)
    fb, fk = _to_fock(space, bra, basis), _to_fock(space, ket, basis)
    for idx in np.ndindex(*(n,) * 6):
        p, q, r, s, t, u = idx
        ref = fb @ (E[p, q] @ (E[r, s] @ (E[t, u] @ fk)))
        assert abs(G3[idx] - ref) < 1e-12, idx


def test_rdm3_trace_and_picks():
    n, na, nb = 4, 2, 2
    space = fci.DetSpace(n, na, nb)
    rng = np.random.default_rng(6)
    bra, ket = rng.normal(size=(2,) + space.shape)
    G3 = fci.rdm3(space, bra, ket)
    g, G = fci.trdm12(space, bra, ket)
    EE = G + np.einsum("qr,ps->pqrs", np.eye(n), g)
    assert np.abs(np.einsum("pqrstt->pqrs", G3) - (na + nb) * EE).max() < 1e-11
    picks = [(0, 1, 2, 3, 1, 0), (3, 3, 0, 2, 2, 1)]
    assert np.allclose(fci.rdm3(space, bra, ket, picks), [G3[x] for x in picks], atol=1e-13)
