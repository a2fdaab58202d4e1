"""Pins of the determinant FCI oracle against things other than itself."""
from math import comb

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import fci, fock


def _rand_problem(n, nq, seed):
    h, B, _ = synth.make_hamiltonian(n, nq, seed)
    return h, B


def test_colex_order_small():
    # colex order of 2-subsets of {0..3}: {0,1},{0,2},{1,2},{0,3},{1,3},{2,3}
    s = fci.strings(4, 2)
    expect = [0b0011, 0b0101, 0b0110, 0b1001, 0b1010, 0b1100]
    assert list(s) == expect
    for n in range(1, 8):
        for k in range(0, n + 1):
            st = fci.strings(n, k)
            assert len(st) == comb(n, k)
            assert len(set(st.tolist())) == comb(n, k)


@pytest.mark.parametrize("n,na,nb,nq,seed", [(3, 2, 1, 4, 3), (4, 2, 2, 6, 5), (5, 3, 2, 5, 7)])
def test_fci_matches_bruteforce_fock(n, na, nb, nq, seed):
    h, B = _rand_problem(n, nq, seed)
    space = fci.DetSpace(n, na, nb)
    H = fci.dense_hamiltonian(space, h, fci.eri(B), 0.3)
    basis = np.array([int(a) | (int(b) << n) for a in space.sa for b in space.sb])
    Hf = fock.hamiltonian(h, B, basis, fock.alpha_first_positions(n), 0.3).toarray()
    assert np.max(np.abs(H - Hf)) < 1e-12
    assert np.max(np.abs(H - H.T)) < 1e-12
    d = fci.diagonal(space, h, fci.eri(B), 0.3).reshape(-1)
    assert np.max(np.abs(d - np.diag(H))) < 1e-12


def test_particle_number_and_sz_conserved_bruteforce():
    n = 3
    h, B = _rand_problem(n, 3, 11)
    full = np.arange(1 << (2 * n))
    H = fock.hamiltonian(h, B, full, fock.alpha_first_positions(n)).toarray()
    na = np.array([bin(s & 7).count("1") for s in full])
    nb = np.array([bin(s >> 3).count("1") for s in full])
    N = np.diag(na + nb).astype(float)
    Sz = np.diag(0.5 * (na - nb))
    assert np.max(np.abs(H @ N - N @ H)) < 1e-12
    assert np.max(np.abs(H @ Sz - Sz @ H)) < 1e-12


def test_free_fermions_closed_form():
    n, na, nb = 6, 3, 2
    h, _ = _rand_problem(n, 1, 2)
    B = np.zeros((0, n, n))
    w, _, _ = fci.solve(n, na, nb, h, B, nroots=1)
    eps = np.linalg.eigvalsh(h)
    assert abs(w[0] - (eps[:na].sum() + eps[:nb].sum())) < 1e-12


@pytest.mark.parametrize("t,U", [(1.0, 4.0), (0.3, 2.5), (1.0, 0.0)])
def test_hubbard_dimer_closed_form(t, U):
    h = np.array([[0.0, -t], [-t, 0.0]])
    B = np.zeros((2, 2, 2))
    B[0, 0, 0] = np.sqrt(U)
    B[1, 1, 1] = np.sqrt(U)
    w, _, _ = fci.solve(2, 1, 1, h, B, nroots=1)
    assert abs(w[0] - (U - np.sqrt(U * U + 16 * t * t)) / 2) < 1e-12


def test_sigma_hermitian_and_davidson_vs_eigsh():
    n, na, nb = 6, 3, 3
    h, B = _rand_problem(n, 10, 4)
    space = fci.DetSpace(n, na, nb)
    g = fci.eri(B)
    rng = np.random.default_rng(0)
    x, y = rng.standard_normal((2, space.size))
    hx = fci.sigma(space, h, g, x).reshape(-1)
    hy = fci.sigma(space, h, g, y).reshape(-1)
    assert abs(x @ hy - y @ hx) < 1e-11 * np.linalg.norm(hx) * np.linalg.norm(y)
    op = spla.LinearOperator((space.size,) * 2, matvec=lambda v: fci.sigma(space, h, g, v).reshape(-1),
                             dtype=float)
    ev = np.sort(spla.eigsh(op, k=3, which="SA", tol=1e-12)[0])
    d = fci.diagonal(space, h, g).reshape(-1)
    th, _ = fci.davidson(lambda v: fci.sigma(space, h, g, v).reshape(-1), d, 3, tol=1e-9)
    assert np.max(np.abs(th - ev)) < 1e-10
    H = fci.dense_hamiltonian(space, h, g)
    assert np.max(np.abs(np.linalg.eigvalsh(H)[:3] - ev)) < 1e-10


def test_s_squared_integral_on_eigenstates():
    n, na, nb = 4, 2, 2
    h, B = _rand_problem(n, 6, 8)
    w, vs, space = fci.solve(n, na, nb, h, B, nroots=6)
    for c in vs:
        s2 = fci.s_squared(space, c)
        S = (-1 + np.sqrt(1 + 4 * s2)) / 2
        assert abs(S - round(S)) < 1e-9, s2
    # a closed-shell single determinant (orbital 0 doubly occupied, 1 doubly) is a singlet
    c = np.zeros(space.shape)
    c[0, 0] = 1.0
    assert abs(fci.s_squared(space, c)) < 1e-14
    # open-shell triplet component: (a0 b1 - b0 a1)/sqrt2 is a singlet, (+) is a triplet
    space2 = fci.DetSpace(2, 1, 1)
    c = np.zeros(space2.shape)
    ia = {int(s): i for i, s in enumerate(space2.sa)}
    # (a+_0a a+_1b -/+ a+_0b a+_1a)/sqrt2 |0>: since a+_0b a+_1a = -a+_1a a+_0b, the
    # singlet has equal determinant amplitudes and the M_s = 0 triplet opposite ones
    c[ia[1], ia[2]] = 1 / np.sqrt(2)
    c[ia[2], ia[1]] = 1 / np.sqrt(2)
    assert abs(fci.s_squared(space2, c)) < 1e-12
    c[ia[2], ia[1]] = -1 / np.sqrt(2)
    assert abs(fci.s_squared(space2, c) - 2.0) < 1e-12


def test_rdm_identities_and_euler():
    n, na, nb = 5, 3, 2
    h, B = _rand_problem(n, 7, 9)
    w, vs, space = fci.solve(n, na, nb, h, B, nroots=1)
    gamma, Gp = fci.rdm12(space, vs[0])
    N = na + nb
    assert abs(np.trace(gamma) - N) < 1e-12
    assert np.max(np.abs(np.einsum("pqrr->pq", Gp) - (N - 1) * gamma)) < 1e-12
    assert np.max(np.abs(Gp - Gp.transpose(2, 3, 0, 1))) < 1e-12
    assert abs(fci.energy_from_rdm(h, B, gamma, Gp) - w[0]) < 1e-12
    dh, dB = fci.integral_gradients(B, gamma, Gp)
    # E is homogeneous of degree 1 in h and 2 in B (e_core = 0)
    assert abs(np.sum(h * dh) + 0.5 * np.sum(B * dB) - w[0]) < 1e-12


def test_integral_gradient_finite_difference():
    n, na, nb = 4, 2, 2
    h, B = _rand_problem(n, 5, 12)
    w, vs, space = fci.solve(n, na, nb, h, B, nroots=2)
    rng = np.random.default_rng(3)
    # directions must keep h and every B^Q symmetric (H is Hermitian only then)
    dh_dir = rng.standard_normal(h.shape)
    dh_dir = dh_dir + dh_dir.T
    dB_dir = rng.standard_normal(B.shape)
    dB_dir = dB_dir + dB_dir.transpose(0, 2, 1)
    eps = 1e-5
    for root in range(2):
        gamma, Gp = fci.rdm12(space, vs[root])
        gh, gB = fci.integral_gradients(B, gamma, Gp)
        ep = fci.solve(n, na, nb, h + eps * dh_dir, B + eps * dB_dir, nroots=2)[0][root]
        em = fci.solve(n, na, nb, h - eps * dh_dir, B - eps * dB_dir, nroots=2)[0][root]
        fd = (ep - em) / (2 * eps)
        an = np.sum(gh * dh_dir) + np.sum(gB * dB_dir)
        assert abs(fd - an) < 1e-7
