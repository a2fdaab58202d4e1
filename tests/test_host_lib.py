"""Host-side tests of the C-ABI library (no GPU calls): symbols, validation, MPO."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
from oracle import fock

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    import paper_2609_09990_amd as pk
    return pk


def test_library_exports_every_header_symbol():
    pk = _lib()
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"^\s*(?:[\w\*]+\s+)+\**(dmrg_\w+)\s*\(", txt, re.M))
    assert len(names) >= 15
    raw = ctypes.CDLL(pk.LIB_PATH)
    missing = [n for n in sorted(names) if not hasattr(raw, n)]
    assert not missing, missing


def test_problem_validation():
    pk = _lib()
    h, B, _ = synth.make_hamiltonian(4, 3, 0)
    bad = h.copy()
    bad[0, 1] += 1e-6
    with pytest.raises(pk.DMRGError) as e:
        pk.Problem(bad, B, 2, 2)
    assert e.value.code == -1
    Bb = B.copy()
    Bb[1, 0, 2] += 1e-6
    with pytest.raises(pk.DMRGError) as e:
        pk.Problem(h, Bb, 2, 2)
    assert e.value.code == -1
    with pytest.raises(pk.DMRGError) as e:
        pk.Problem(h, B, 5, 2)
    assert e.value.code == -5


def _dense_mpo(prob):
    n = prob.n
    dims = prob.mpo_dims()
    T = np.zeros((dims[0], 1, 1))
    T[0, 0, 0] = 1.0
    for k in range(n):
        a, b, c, op = prob.mpo_site(k)
        Tn = np.zeros((dims[k + 1], T.shape[1] * 4, T.shape[2] * 4))
        for i in range(len(a)):
            Tn[b[i]] += c[i] * np.kron(T[a[i]], op[i])
        T = Tn
    assert T.shape[0] == 1
    return T[0]


@pytest.mark.parametrize("n,nq,seed", [(2, 2, 1), (3, 3, 2), (4, 4, 3), (5, 3, 4), (4, 0, 5)])
def test_mpo_contracts_to_fock_hamiltonian(n, nq, seed):
    """The Cholesky-channel MPO, contracted densely, equals the brute-force
    Jordan-Wigner Hamiltonian in the site-product basis (all particle numbers)."""
    pk = _lib()
    h, B, _ = synth.make_hamiltonian(n, nq, seed)
    prob = pk.Problem(h, B, n // 2, n - n // 2)
    Hm = _dense_mpo(prob)
    Hf = fock.hamiltonian(h, B, fock.site_product_basis(n), fock.interleaved_positions(n)).toarray()
    assert np.max(np.abs(Hm - Hf)) < 1e-12


def test_mpo_bond_dimensions_at_scale():
    """Channel count at the middle cut: I, H, 4L one-fermion, N_Q Cholesky and
    8 n^2 pair channels (n orbitals on the smaller side), minus edge pruning."""
    pk = _lib()
    n, nq = 12, 64
    h, B, _ = synth.make_hamiltonian(n, nq, 0)
    d = pk.Problem(h, B, 6, 6).mpo_dims()
    assert d[0] == 1 and d[-1] == 1
    full = 2 + 4 * n + nq + 8 * 36
    assert 2 + 4 * n + nq < d[6] <= full
    assert d[6] == max(d)


def test_mpo_keeps_structure_of_exact_zero_integrals():
    """Integrals that are exactly zero add nothing to H, yet their entries stay
    in the MPO (their derivative is generally non-zero): the dense contraction
    still equals the brute-force Hamiltonian and the channel counts equal those
    of a generic Hamiltonian of the same shape."""
    pk = _lib()
    n, nq = 5, 3
    h, B, _ = synth.make_hamiltonian(n, nq, 6)
    ref_dims = pk.Problem(h, B, 3, 2).mpo_dims()
    h[0, 3] = h[3, 0] = 0.0
    h[1, 1] = 0.0
    B[0, 0, 4] = B[0, 4, 0] = 0.0
    B[2] = 0.0
    prob = pk.Problem(h, B, 3, 2)
    Hf = fock.hamiltonian(h, B, fock.site_product_basis(n), fock.interleaved_positions(n)).toarray()
    assert np.max(np.abs(_dense_mpo(prob) - Hf)) < 1e-12
    assert list(prob.mpo_dims()) == list(ref_dims)


def test_fiedler_order_matches_oracle():
    """dmrg_fiedler_order (host only) against the oracle's numpy eigenvector on
    random symmetric non-negative matrices and a shuffled path graph."""
    import paper_2609_09990_amd as pk
    from oracle import orbital
    rng = np.random.default_rng(4)
    for n in (2, 5, 12, 20):
        I = rng.uniform(0, 1, size=(n, n))
        I = I + I.T
        np.fill_diagonal(I, 0)
        order, v = pk.fiedler_order(I)
        ref_order, ref_v = orbital.fiedler_order(I)
        assert np.abs(v - ref_v).max() < 1e-10
        assert list(order) == list(ref_order)
    perm = np.array([3, 0, 6, 2, 5, 1, 4])
    I = np.zeros((7, 7))
    for k in range(6):
        I[perm[k], perm[k + 1]] = I[perm[k + 1], perm[k]] = 1.0
    order, _ = pk.fiedler_order(I)
    assert list(order) in (list(perm), list(perm[::-1]))


def test_ci_dimensions_and_length_refusals():
    """The CI matrix shape is (C(n, n_alpha), C(n, n_beta)), and every call on
    device CI vectors refuses a length other than their product with
    DMRG_EINVAL before any device work (the vector pointers below are never
    dereferenced: the host check comes first)."""
    from math import comb
    pk = _lib()
    h, B, _ = synth.make_hamiltonian(6, 3, 0)
    prob = pk.Problem(h, B, 4, 2)
    assert prob.ci_dims() == (comb(6, 4), comb(6, 2))
    n = comb(6, 4) * comb(6, 2)
    fake = ctypes.c_void_p(1 << 20)
    host = np.zeros(6 ** 6)
    hp = host.ctypes.data_as(ctypes.c_void_p)
    calls = {
        "dmrg_ci_rdm12": lambda m: pk.dmrg_ci_rdm12(prob.h, m, fake, fake, hp, hp, hp, None),
        "dmrg_ci_apply_v": lambda m: pk.dmrg_ci_apply_v(prob.h, m, fake, ctypes.c_void_p(2 << 20), None),
        "dmrg_ci_rdm3": lambda m: pk.dmrg_ci_rdm3(prob.h, m, fake, fake, hp, None),
        "dmrg_orbital_rdm2": lambda m: pk.dmrg_orbital_rdm2(prob.h, m, fake, hp, None),
        "dmrg_mutual_information": lambda m: pk.dmrg_mutual_information(prob.h, m, fake, hp, hp, None),
    }
    for name, call in calls.items():
        for m in (0, n - 1, n + 1, -n):
            assert call(m) == -1, (name, m)
            assert b"CI dimension" in pk.dmrg_last_error(), name


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: asked for several it exits with status 2 and
    says why, before touching any device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
