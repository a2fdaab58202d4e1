"""Pins of the oracle's own MPO and block-sparse two-site H_eff (oracle.mpo,
oracle.blocks): against the brute-force Fock-space Hamiltonian and the
projected FCI sigma, which use neither an MPO nor environments."""
import numpy as np
import pytest

import synth
from oracle import blocks, embed, fock
from oracle import mpo as om


@pytest.mark.parametrize("n,nq,seed,mode", [(2, 3, 0, "full"), (3, 4, 1, "full"), (4, 5, 2, "full"),
                                            (3, 0, 3, "one-body"), (3, 4, 4, "two-body"),
                                            (4, 2, 5, "sparse")])
def test_mpo_contracts_to_bruteforce_hamiltonian(n, nq, seed, mode):
    """The automaton MPO contracted densely equals the Jordan-Wigner Fock H (all particle numbers)."""
    h, B, _ = synth.make_hamiltonian(n, max(nq, 1), seed)
    if mode == "one-body":
        B = np.zeros((0, n, n))
    elif mode == "two-body":
        h = np.zeros_like(h)
    elif mode == "sparse":  # exactly-zero integrals: their terms vanish, the rest must stay exact
        h[0, n - 1] = h[n - 1, 0] = 0.0
        B[:, 1, :] = 0.0
        B[:, :, 1] = 0.0
    m = om.build_mpo(h, B)
    H = fock.hamiltonian(h, B if B.size else np.zeros((1, n, n)), fock.site_product_basis(n),
                         fock.interleaved_positions(n)).toarray()
    D = om.dense(m)
    assert np.max(np.abs(D - H)) <= 1e-12 * max(1.0, np.max(np.abs(H)))
    assert m.dims()[0] == 1 and m.dims()[-1] == 1


def test_mpo_bond_dimension_is_pairs_plus_singles():
    """At a cut c <= L/2 of an n-orbital chain the channels are I, D, the 4c single
    operators on the left, the ladder pairs on the left and the 4(n-c) single
    operators carried on the right (a count from the construction's rule)."""
    n = 6
    h, B, _ = synth.make_hamiltonian(n, 8, 7)
    m = om.build_mpo(h, B)
    c = 2
    modes = 2 * c  # spin orbitals left of the cut
    pairs_diff_site = 16 * (c * (c - 1) // 2)  # two ladder ops on two different sites
    pairs_same_site = 6 * c                    # canonical same-site pairs
    expect = 2 + 2 * modes + pairs_diff_site + pairs_same_site + 4 * (n - c)
    assert m.dims()[c] == expect


@pytest.mark.parametrize("n,na,nb,nq,M,k", [(4, 2, 2, 5, 16, 1), (5, 3, 2, 6, 8, 0), (6, 3, 3, 8, 20, 2),
                                            (6, 3, 3, 8, 20, 4), (7, 4, 3, 6, 12, 3), (8, 4, 4, 10, 30, 3),
                                            (6, 3, 3, 8, 64, 2)])
def test_block_sigma_equals_projected_fci_sigma(n, na, nb, nq, M, k):
    """sigma through the oracle's MPO and environments equals P^T H P psi (determinant space)."""
    h, B, _ = synth.make_hamiltonian(n, nq, 1)
    m = om.build_mpo(h, B)
    mps = synth.random_mps(n, na, nb, M, seed=3)
    psi = synth.random_twosite(mps["bonds"], k, seed=4)
    ts = blocks.TwoSite(m, mps, k)
    fl = [0.0]
    got = ts.sigma(psi, flops=fl)
    ref = embed.sigma_twosite(h, B, mps, k, psi, na, nb)
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)
    assert fl[0] > 0
    # sampled blocks are the same numbers as the full evaluation
    out = ts.output_blocks()
    pick = [out[0], out[len(out) // 2], out[-1]]
    part = ts.sigma(psi, blocks=pick)
    full = blocks.unpack(ts.bl, ts.br, blocks.twosite_qn(), got)
    for key in pick:
        assert np.array_equal(part[key], full[key])


@pytest.mark.parametrize("n,na,nb,M,k", [(4, 2, 2, 6, 1), (5, 2, 3, 5, 2)])
def test_block_diag_and_symmetry(n, na, nb, M, k):
    """diag(H_eff) equals the diagonal of the dense P^T H P from unit vectors; H_eff is symmetric."""
    h, B, _ = synth.make_hamiltonian(n, 4, 9)
    m = om.build_mpo(h, B)
    mps = synth.random_mps(n, na, nb, M, seed=11)
    ts = blocks.TwoSite(m, mps, k)
    size = synth.tensor_size(mps["bonds"][k], mps["bonds"][k + 2], synth.twosite_qn())
    H = np.zeros((size, size))
    for i in range(size):
        e = np.zeros(size)
        e[i] = 1.0
        H[:, i] = embed.sigma_twosite(h, B, mps, k, e, na, nb)
    assert np.max(np.abs(ts.diag() - np.diag(H))) <= 1e-13 * np.max(np.abs(H))
    x = synth.random_twosite(mps["bonds"], k, seed=1)
    y = synth.random_twosite(mps["bonds"], k, seed=2)
    assert abs(x @ ts.sigma(y) - y @ ts.sigma(x)) <= 1e-13 * np.max(np.abs(H))


def test_slab_pack_roundtrip():
    mps = synth.random_mps(6, 3, 3, 10, seed=2)
    bl, br = blocks.Bond(mps["bonds"][2]), blocks.Bond(mps["bonds"][4])
    v = synth.random_twosite(mps["bonds"], 2, seed=3)
    assert np.array_equal(blocks.pack(bl, br, blocks.twosite_qn(), blocks.unpack(bl, br, blocks.twosite_qn(), v)), v)
