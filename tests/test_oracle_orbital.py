"""Pins of the oracle's orbital entanglement (oracle.orbital): two-orbital
density matrices against expectation values of |t><s| built from brute-force
Fock-space ladder operators, a determinant, the two-orbital singlet, traces and
partial traces, and the Fiedler vector of a path graph.  CPU only."""
import numpy as np
import pytest

from oracle import fci, fock, orbital


def _to_fock(space, C, basis):
    n = space.n
    ia = {int(s): i for i, s in enumerate(space.sa)}
    ib = {int(s): i for i, s in enumerate(space.sb)}
    mask = (1 << n) - 1
    return np.array([C[ia[int(s) & mask], ib[int(s) >> n]] for s in basis])


def _ketbra_expectation(n, basis, psi, i, j, t, s):
    """<Psi| C_s P_0 C_t^+ |Psi> with C_x the creators of local state x in the
    local order (i a, j a, i b, j b) and P_0 the projector on the local vacuum:
    the element rho[t, s] of the two-orbital density matrix."""
    pos = fock.alpha_first_positions(n)
    below = fock._below_masks(pos)
    loc = [i, j, n + i, n + j]

    def occ_of(x):
        si, sj = x % 4, x // 4
        bits = [si & 1, sj & 1, si >> 1, sj >> 1]
        return [loc[t_] for t_ in range(4) if bits[t_]]

    st = np.asarray(basis, dtype=np.int64)
    sg = np.ones(len(st), dtype=np.int64)
    # C_t^+ : annihilators of t's local spin orbitals, last creator first undone
    for so in occ_of(t)[::-1][::-1]:
        st, sg = fock._ladder(st, sg, so, False, below)
    # P_0: every local spin orbital empty
    for so in loc:
        sg = np.where((st >> so) & 1, 0, sg)
    for so in occ_of(s)[::-1]:
        st, sg = fock._ladder(st, sg, so, True, below)
    index = {int(b): k for k, b in enumerate(basis)}
    val = 0.0
    for k in np.nonzero(sg)[0]:
        if int(st[k]) in index:  # |t>, |s> of different electron counts leave the sector
            val += psi[index[int(st[k])]] * sg[k] * psi[k]
    return val


@pytest.mark.parametrize("n,na,nb,i,j", [(3, 2, 1, 0, 2), (3, 1, 1, 0, 1), (4, 2, 2, 1, 3), (4, 2, 1, 0, 3)])
def test_two_orbital_rdm_equals_fock_space_ketbras(n, na, nb, i, j):
    space = fci.DetSpace(n, na, nb)
    rng = np.random.default_rng(n * 31 + i * 7 + j)
    C = rng.normal(size=space.shape)
    C /= np.linalg.norm(C)
    rho = orbital.orbital_rdm(space, C, [i, j])
    basis = fock.sector_basis(n, na, nb)
    psi = _to_fock(space, C, basis)
    for t in range(16):
        for s in range(16):
            ref = _ketbra_expectation(n, basis, psi, i, j, t, s)
            assert abs(rho[t, s] - ref) < 1e-12, (t, s, rho[t, s], ref)


def test_determinant_and_singlet_pair():
    space = fci.DetSpace(3, 2, 1)
    C = np.zeros(space.shape)
    C[1, 2] = 1.0
    s1, I = orbital.mutual_information(space, C)
    assert np.abs(s1).max() < 1e-12 and np.abs(I).max() < 1e-12
    # two orbitals, one pair: (|2 0> + |0 2>) / sqrt 2
    space = fci.DetSpace(2, 1, 1)
    C = np.zeros(space.shape)
    C[0, 0] = C[1, 1] = 1 / np.sqrt(2)
    s1, I = orbital.mutual_information(space, C)
    assert np.allclose(s1, np.log(2)) and abs(I[0, 1] - np.log(2)) < 1e-12
    assert abs(orbital.entropy(orbital.orbital_rdm(space, C, [0, 1]))) < 1e-12


def test_traces_and_partial_traces():
    space = fci.DetSpace(4, 2, 2)
    C = np.random.default_rng(2).normal(size=space.shape)
    r2 = orbital.orbital_rdm(space, C, [1, 2])
    r1 = orbital.orbital_rdm(space, C, [1])
    assert abs(np.trace(r2) - 1) < 1e-12 and np.linalg.eigvalsh(r2).min() > -1e-12
    part = np.einsum("jaja->a", r2.reshape(4, 4, 4, 4))  # L = s_i + 4 s_j: sum over s_j
    assert np.abs(np.diag(r1) - part).max() < 1e-12
    assert np.abs(r1 - np.diag(np.diag(r1))).max() < 1e-14  # number and S_z conserving


def test_fiedler_order_of_a_shuffled_path():
    """A path graph with its vertices shuffled: the Fiedler ordering walks the
    path from one end to the other."""
    n = 7
    perm = np.array([3, 0, 6, 2, 5, 1, 4])
    I = np.zeros((n, n))
    for k in range(n - 1):
        a, b = perm[k], perm[k + 1]
        I[a, b] = I[b, a] = 1.0
    order, v = orbital.fiedler_order(I)
    assert list(order) == list(perm) or list(order) == list(perm[::-1])
