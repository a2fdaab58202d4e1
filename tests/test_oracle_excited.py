"""Pins of the oracle pieces behind excited states (Sec. II.F): the sparse
<S^2>, the projection of a lower state into a two-site space and the MPS
overlap.  CPU only."""
import numpy as np
import pytest

import synth
from oracle import blocks, embed, fci


@pytest.mark.parametrize("n,na,nb", [(4, 2, 2), (5, 3, 2), (5, 2, 3), (4, 3, 0), (3, 3, 1), (5, 1, 1)])
def test_sparse_s_squared_equals_determinant_loops(n, na, nb):
    """Brute force: the per-determinant ladder loops give the same <S^2>."""
    space = fci.DetSpace(n, na, nb)
    rng = np.random.default_rng(n * 100 + na * 10 + nb)
    for _ in range(3):
        c = rng.normal(size=space.shape)
        a = fci.s_squared_sparse(space, c)
        b = fci.s_squared(space, c)
        assert abs(a - b) <= 1e-12 * max(1.0, abs(b)), (a, b)


def test_sparse_s_squared_closed_forms():
    # eigenstates of a spin-free H have <S^2> = S(S+1)
    h, B, _ = synth.make_hamiltonian(5, 6, 4)
    w, vs, space = fci.solve(5, 3, 2, h, B, nroots=6)
    for c in vs:
        s2 = fci.s_squared_sparse(space, c)
        two_s = -1 + np.sqrt(1 + 4 * s2)  # 2S from S(S+1)
        assert abs(two_s - round(two_s)) < 1e-9, s2
        assert round(two_s) % 2 == 1  # S_z = 1/2 sector: doublets, quartets, ...
    # the fully polarised determinant: S = S_z = n_alpha / 2
    space = fci.DetSpace(4, 3, 0)
    c = np.zeros(space.shape)
    c[0, 0] = 1.0
    assert abs(fci.s_squared_sparse(space, c) - 1.5 * 2.5) < 1e-14
    # two electrons in two orbitals: equal amplitudes of (a0 b1) and (a1 b0) is
    # the singlet, opposite amplitudes the M_s = 0 triplet
    space = fci.DetSpace(2, 1, 1)
    ia = {int(s): i for i, s in enumerate(space.sa)}
    c = np.zeros(space.shape)
    c[ia[1], ia[2]] = c[ia[2], ia[1]] = 1 / np.sqrt(2)
    assert abs(fci.s_squared_sparse(space, c)) < 1e-12
    c[ia[2], ia[1]] = -1 / np.sqrt(2)
    assert abs(fci.s_squared_sparse(space, c) - 2.0) < 1e-12


def _explicit_basis(mps, k):
    A = embed.site_tensors(mps)
    U = embed.left_basis(A, k)
    V = embed.right_basis(A, k + 2)
    cols = []
    for a in range(U.shape[1]):
        for s1 in range(4):
            for s2 in range(4):
                for b in range(V.shape[1]):
                    e1 = np.zeros(4)
                    e1[s1] = 1
                    e2 = np.zeros(4)
                    e2[s2] = 1
                    cols.append(np.kron(np.kron(np.kron(U[:, a], e1), e2), V[:, b]))
    return np.array(cols).T, U.shape[1], V.shape[1]


@pytest.mark.parametrize("n,na,nb,M,k", [(4, 2, 2, 3, 1), (4, 2, 1, 2, 0), (5, 3, 2, 4, 2), (5, 2, 2, 3, 3)])
def test_projection_vs_explicit_basis(n, na, nb, M, k):
    """phi = P^T Phi with P's columns |a s1 s2 b> built one by one."""
    psi = synth.random_mps(n, na, nb, M, seed=5)
    phi_mps = synth.random_mps(n, na, nb, M + 1, seed=9)
    got = embed.project_twosite(psi, k, phi_mps)
    P, Dl, Dr = _explicit_basis(psi, k)
    full = embed.left_basis(embed.site_tensors(phi_mps), n).reshape(-1)
    ref = (P.T @ full).reshape(Dl, 16, Dr)
    ref = embed.dense_to_slab(psi["bonds"][k], psi["bonds"][k + 2], embed.twosite_qn(), ref)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def _right_canonical(mps):
    """Right-canonical form of an MPS (QR of each site's transpose from the right),
    the state unchanged up to the norm carried into site 0."""
    bonds = mps["bonds"]
    n = len(mps["sites"])
    A = embed.site_tensors(mps)
    for k in range(n - 1, 0, -1):
        D0, _, D1 = A[k].shape
        Q, R = np.linalg.qr(A[k].reshape(D0, 4 * D1).T)
        A[k] = Q.T.reshape(-1, 4, D1)
        A[k - 1] = np.einsum("asb,cb->asc", A[k - 1], R)
    return A, bonds


def test_projection_of_the_state_itself():
    """Closed form: with sites 2.. right-orthonormal the step-0 basis is
    orthonormal, so projecting the state into its own step-0 space returns its
    two-site tensor, and projecting another state cannot increase its norm."""
    n, na, nb = 5, 3, 2
    mps = synth.random_mps(n, na, nb, 64, seed=3)  # full bonds: QR keeps the sectors
    A, bonds = _right_canonical(mps)
    sites = [embed.dense_to_slab(bonds[k], bonds[k + 1], embed.SITE_QN, A[k]) for k in range(n)]
    rc = {"bonds": bonds, "sites": sites}
    got = embed.project_twosite(rc, 0, rc)
    two = blocks.twosite_from_sites(rc, 0)
    assert np.linalg.norm(got - two) <= 1e-12 * np.linalg.norm(two)
    full = embed.left_basis(embed.site_tensors(rc), n).reshape(-1)
    assert abs(np.linalg.norm(full) - np.linalg.norm(two)) <= 1e-12 * np.linalg.norm(two)
    other = synth.random_mps(n, na, nb, 3, seed=8)
    p = embed.project_twosite(rc, 0, other)
    f = embed.left_basis(embed.site_tensors(other), n).reshape(-1)
    assert np.linalg.norm(p) <= np.linalg.norm(f) * (1 + 1e-12)


def test_overlap_properties():
    n, na, nb = 5, 2, 3
    a = synth.random_mps(n, na, nb, 4, seed=1)
    b = synth.random_mps(n, na, nb, 6, seed=2)
    assert abs(embed.overlap(a, a) - 1.0) < 1e-14
    o = embed.overlap(a, b)
    assert abs(o) <= 1.0
    # the determinant map is a signed permutation: the CI vectors give the same overlap
    ca = embed.mps_state(a, na, nb).reshape(-1)
    cb = embed.mps_state(b, na, nb).reshape(-1)
    assert abs(o - ca @ cb / np.linalg.norm(ca) / np.linalg.norm(cb)) < 1e-13
