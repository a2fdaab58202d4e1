"""Orbital entanglement on the GPU (Sec. II.H ordering) through the C ABI,
against the CPU oracle: two-orbital density matrices of every pair element-wise,
one-orbital entropies and mutual information, and the Fiedler order of a
DMRG state's mutual information after shuffling the orbitals."""
import numpy as np
import pytest

import synth
from oracle import fci, orbital

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("n,na,nb", [(2, 1, 1), (4, 2, 2), (5, 3, 2), (6, 3, 3), (7, 2, 4)])
def test_orbital_rdm2_and_mutual_information_match_oracle(n, na, nb):
    torch = _torch()
    import paper_2609_09990_amd as pk
    print(f"orbital rdm n={n} ({na},{nb})", flush=True)
    h, B, e0 = synth.make_hamiltonian(n, 4, 0)
    prob = pk.Problem(h, B, na, nb, e0)
    space = fci.DetSpace(n, na, nb)
    c = np.random.default_rng(n * 13 + na).normal(size=space.shape)
    dc = torch.from_numpy(c).cuda()
    rho = prob.orbital_rdm2(dc)
    p = 0
    for i in range(n):
        for j in range(i + 1, n):
            ref = orbital.orbital_rdm(space, c, [i, j])
            assert np.abs(rho[p] - ref).max() <= 1e-12, (i, j)
            p += 1
    s1, I = prob.mutual_information(dc)
    rs1, rI = orbital.mutual_information(space, c)
    assert np.abs(s1 - rs1).max() <= 1e-10 and np.abs(I - rI).max() <= 1e-10


def test_fiedler_order_of_a_dmrg_state_cas8():
    """CAS(8,8), N_Q = 32 with its orbitals shuffled: a DMRG state at M = 32,
    its CI vector, mutual information and Fiedler order equal the oracle's from
    the same CI vector; the energies of M = 32 runs in the shuffled and the
    Fiedler order are printed."""
    torch = _torch()
    import paper_2609_09990_amd as pk
    h, B, e0 = synth.make_hamiltonian(8, 32, 0)
    perm = np.array([5, 2, 7, 0, 3, 6, 1, 4])
    hs, Bs = pk.reorder_integrals(h, B, perm)
    prob = pk.Problem(hs, Bs, 4, 4, e0)
    sol = pk.Solver(prob, M=32, tol=1e-9)
    e_shuf = sol.sweep(4)[0][0]
    c = sol.mps_to_ci()
    s1, I = prob.mutual_information(c)
    order, v = pk.fiedler_order(I)
    space = fci.DetSpace(8, 4, 4)
    rs1, rI = orbital.mutual_information(space, c.cpu().numpy())
    ref_order, _ = orbital.fiedler_order(rI)
    assert np.abs(I - rI).max() <= 1e-10
    assert list(order) == list(ref_order)
    ho, Bo = pk.reorder_integrals(hs, Bs, order)
    e_ord = pk.Solver(pk.Problem(ho, Bo, 4, 4, e0), M=32, tol=1e-9).sweep(4)[0][0]
    print(f"M=32: shuffled order E {e_shuf:.8f}, Fiedler order {list(order)} E {e_ord:.8f}", flush=True)


@pytest.mark.parametrize("n,na,nb,M,seed", [(3, 2, 1, 4, 1), (4, 2, 2, 16, 2), (5, 3, 2, 8, 3), (6, 3, 3, 12, 4),
                                            (7, 4, 2, 20, 5)])
def test_mps_orbital_rdm2_matches_oracle(n, na, nb, M, seed):
    """Two-orbital density matrices from the MPS itself (pair MPO and the
    gradient contractions) against the oracle's on the MPS's CI vector, every
    element, for MPS in no canonical form (truncated, ragged bonds)."""
    _torch()
    import paper_2609_09990_amd as pk
    print(f"mps orbital rdm n={n} ({na},{nb}) M={M}", flush=True)
    h, B, e0 = synth.make_hamiltonian(n, 4, 0)
    mps = synth.random_mps(n, na, nb, M, seed=seed)
    sol = pk.Solver(pk.Problem(h, B, na, nb, e0), M=M)
    sol.set_mps(mps["bonds"], mps["sites"])
    rho, s1, I = sol.orbital_entanglement()
    from oracle import embed
    space = fci.DetSpace(n, na, nb)
    c = embed.mps_state(mps, na, nb)
    p = 0
    for i in range(n):
        for j in range(i + 1, n):
            ref = orbital.orbital_rdm(space, c, [i, j])
            assert np.abs(rho[p] - ref).max() <= 1e-12, (i, j, np.abs(rho[p] - ref).max())
            p += 1
    rs1, rI = orbital.mutual_information(space, c)
    assert np.abs(s1 - rs1).max() <= 1e-10 and np.abs(I - rI).max() <= 1e-10


def test_mps_and_ci_routes_agree_cas10():
    """CAS(10,10), N_Q = 16 after two sweeps at M = 64: the MPS route and the CI
    route give the same density matrices, entropies and mutual information."""
    _torch()
    import paper_2609_09990_amd as pk
    h, B, e0 = synth.make_hamiltonian(10, 16, 2)
    prob = pk.Problem(h, B, 5, 5, e0)
    sol = pk.Solver(prob, M=64, tol=1e-8)
    sol.sweep(2)
    rho, s1, I = sol.orbital_entanglement()
    c = sol.mps_to_ci()
    rho_ci = prob.orbital_rdm2(c)
    s1_ci, I_ci = prob.mutual_information(c)
    print(f"max |rho diff| {np.abs(rho - rho_ci).max():.1e}, max I {I.max():.3f}", flush=True)
    assert np.abs(rho - rho_ci).max() <= 1e-11
    assert np.abs(s1 - s1_ci).max() <= 1e-10 and np.abs(I - I_ci).max() <= 1e-10


def test_mps_orbital_entanglement_properties_cas16():
    """CAS(16,16), N_Q = 32 at M = 128 (CI vector of 1.7e8 determinants: the
    MPS route only): every two-orbital density matrix is symmetric, positive
    semi-definite with unit trace and its one-orbital partial traces agree
    between pairs; entropies and mutual information are non-negative and the
    Fiedler order is a permutation."""
    _torch()
    import paper_2609_09990_amd as pk
    h, B, e0 = synth.make_hamiltonian(16, 32, 1)
    sol = pk.Solver(pk.Problem(h, B, 8, 8, e0), M=128, tol=1e-7)
    sol.sweep(2)
    rho, s1, I = sol.orbital_entanglement()
    n = 16
    assert np.abs(rho - rho.transpose(0, 2, 1)).max() <= 1e-12
    assert np.abs(np.trace(rho, axis1=1, axis2=2) - 1.0).max() <= 1e-10
    assert min(np.linalg.eigvalsh(r).min() for r in rho) >= -1e-10
    one = {}
    p = 0
    for i in range(n):
        for j in range(i + 1, n):
            d = np.diag(rho[p]).reshape(4, 4)  # [s_j][s_i]
            for o, v in ((i, d.sum(axis=0)), (j, d.sum(axis=1))):
                if o in one:
                    assert np.abs(one[o] - v).max() <= 1e-10
                one[o] = v
            p += 1
    assert s1.min() >= -1e-12 and I.min() >= -1e-10 and np.abs(I - I.T).max() <= 1e-14
    order, _ = pk.fiedler_order(I)
    assert sorted(order) == list(range(n))
    print(f"s1 max {s1.max():.3f}, I max {I.max():.3f}, order {list(order)}", flush=True)
