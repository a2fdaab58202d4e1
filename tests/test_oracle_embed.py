"""Pins of the MPS embedding and the two-site projected sigma."""
import numpy as np
import pytest

import synth
from oracle import embed, fci, fock


@pytest.mark.parametrize("n,na,nb", [(3, 2, 1), (4, 2, 2)])
def test_interleaved_sign_rule(n, na, nb):
    """H in the interleaved (site-product) JW basis equals S H_det S, S = sign rule."""
    h, B, _ = synth.make_hamiltonian(n, 5, 21)
    space = fci.DetSpace(n, na, nb)
    Hd = fci.dense_hamiltonian(space, h, fci.eri(B))
    labels = np.array([int(a) | (int(b) << n) for a in space.sa for b in space.sb])
    Hi = fock.hamiltonian(h, B, labels, fock.interleaved_positions(n)).toarray()
    _, sgn = embed.det_map(n, na, nb)
    s = sgn.reshape(-1)
    assert np.max(np.abs(Hi - s[:, None] * Hd * s[None, :])) < 1e-12
    # and the sign rule matters: without it the matrices differ for n >= 2
    assert np.max(np.abs(Hi - Hd)) > 1e-3


def test_site_product_index_matches_labels():
    n = 3
    sp_basis = fock.site_product_basis(n)
    idx, _ = embed.det_map(n, 2, 1)
    space = fci.DetSpace(n, 2, 1)
    for i, a in enumerate(space.sa):
        for j, b in enumerate(space.sb):
            assert sp_basis[idx[i, j]] == (int(a) | (int(b) << n))


@pytest.mark.parametrize("n,na,nb,M,k", [(4, 2, 2, 3, 1), (4, 2, 1, 2, 0), (5, 3, 2, 4, 2)])
def test_twosite_sigma_vs_bruteforce_projection(n, na, nb, M, k):
    """P^T H P psi with P built densely and H the brute-force interleaved Fock H."""
    h, B, _ = synth.make_hamiltonian(n, 4, 33)
    mps = synth.random_mps(n, na, nb, M, seed=5)
    psi = synth.random_twosite(mps["bonds"], k, seed=6)
    got = embed.sigma_twosite(h, B, mps, k, psi, na, nb)

    A = embed.site_tensors(mps)
    U = embed.left_basis(A, k)
    V = embed.right_basis(A, k + 2)
    Dl, Dr = U.shape[1], V.shape[1]
    # explicit P: columns are |a s1 s2 b> in the site-product basis
    cols = []
    for a in range(Dl):
        for s1 in range(4):
            for s2 in range(4):
                for b in range(Dr):
                    e1 = np.zeros(4); e1[s1] = 1
                    e2 = np.zeros(4); e2[s2] = 1
                    cols.append(np.kron(np.kron(np.kron(U[:, a], e1), e2), V[:, b]))
    P = np.array(cols).T
    Hf = fock.hamiltonian(h, B, fock.site_product_basis(n), fock.interleaved_positions(n)).toarray()
    pd = embed.slab_to_dense(mps["bonds"][k], mps["bonds"][k + 2], embed.twosite_qn(), psi).reshape(-1)
    ref = (P.T @ Hf @ P @ pd).reshape(Dl, 16, Dr)
    ref_flat = embed.dense_to_slab(mps["bonds"][k], mps["bonds"][k + 2], embed.twosite_qn(), ref)
    assert np.linalg.norm(got - ref_flat) <= 1e-12 * np.linalg.norm(ref_flat)


def test_slab_roundtrip():
    mps = synth.random_mps(6, 3, 3, 10, seed=1)
    bonds = mps["bonds"]
    for k in range(5):
        v = synth.random_twosite(bonds, k, seed=k)
        d = embed.slab_to_dense(bonds[k], bonds[k + 2], embed.twosite_qn(), v)
        assert np.allclose(embed.dense_to_slab(bonds[k], bonds[k + 2], embed.twosite_qn(), d), v)
        assert abs(np.linalg.norm(d) - np.linalg.norm(v)) < 1e-12
