"""Adjoint form: integral gradients of the MPS energy (dmrg_grad) on the GPU
against the oracle's reduced-density-matrix contraction of the same state
(gamma and Gamma' of the determinant CI vector, dE/dh = gamma,
dE/dB^Q = sum_rs Gamma'_pqrs B^Q_rs), and against finite differences of the
DMRG energy at full bond."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import embed, fci

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fci_energies.json")


def _pk():
    import paper_2609_09990_amd as pk
    return pk


def _oracle(h, B, c, space, e_core=0.0):
    c = c / np.linalg.norm(c)
    gam, Gp = fci.rdm12(space, c)
    dh, dB = fci.integral_gradients(B, gam, Gp)
    return dh, dB, fci.energy_from_rdm(h, B, gam, Gp, e_core)


@pytest.mark.parametrize("n,na,nb,nq,M", [(2, 1, 1, 2, 4), (4, 2, 2, 5, 16), (5, 3, 2, 4, 10),
                                          (6, 3, 3, 8, 12), (6, 3, 3, 8, 400), (7, 4, 3, 9, 24)])
def test_grad_of_random_mps_matches_oracle_rdm_contraction(n, na, nb, nq, M):
    pk = _pk()
    h, B, e0 = synth.make_hamiltonian(n, nq, 0)
    e0 = 0.75
    sol = pk.Solver(pk.Problem(h, B, na, nb, e0), M=M)
    mps = synth.random_mps(n, na, nb, M, seed=5)
    sol.set_mps(mps["bonds"], mps["sites"])
    dh, dB, e = sol.grad()
    rh, rB, rE = _oracle(h, B, embed.mps_state(mps, na, nb), fci.DetSpace(n, na, nb), e0)
    print(f"n={n} M={M} |dE|={abs(e[0] - rE):.2e} |ddh|={np.abs(dh - rh).max():.2e} "
          f"|ddB|={np.abs(dB - rB).max():.2e}")
    assert abs(e[0] - rE) <= 1e-12 * max(1.0, abs(rE))
    assert np.abs(dh - rh).max() <= 1e-12 * max(1.0, np.abs(rh).max())
    assert np.abs(dB - rB).max() <= 1e-12 * max(1.0, np.abs(rB).max())


def test_grad_with_exact_zero_integrals():
    """Integrals that are exactly zero still get their derivative."""
    pk = _pk()
    n, na, nb, nq, M = 5, 3, 2, 4, 10
    h, B, e0 = synth.make_hamiltonian(n, nq, 0)
    h[0, 3] = h[3, 0] = 0.0
    h[1, 4] = h[4, 1] = 0.0
    h[2, 2] = 0.0
    B[1, 0, 2] = B[1, 2, 0] = 0.0
    B[3, 4, 4] = 0.0
    B[2] = 0.0
    sol = pk.Solver(pk.Problem(h, B, na, nb, e0), M=M)
    mps = synth.random_mps(n, na, nb, M, seed=7)
    sol.set_mps(mps["bonds"], mps["sites"])
    dh, dB, _ = sol.grad()
    rh, rB, _ = _oracle(h, B, embed.mps_state(mps, na, nb), fci.DetSpace(n, na, nb))
    assert abs(rh[0, 3]) > 1e-3 and abs(rB[1, 0, 2]) > 1e-4
    assert np.abs(dh - rh).max() <= 1e-12
    assert np.abs(dB - rB).max() <= 1e-12


def test_grad_full_bond_cas10_matches_fci():
    """CAS(10,10), 48 Cholesky vectors, M = 1024 (exact): the converged ground
    state's gradient equals the FCI one (Hellmann-Feynman, no response)."""
    pk = _pk()
    n, nq = 10, 48
    h, B, e0 = synth.make_hamiltonian(n, nq, 0)
    sol = pk.Solver(pk.Problem(h, B, 5, 5, e0), M=1024, tol=1e-12)
    e, tau, ok = sol.sweep(2)
    dh, dB, eg = sol.grad()
    E, C, space = fci.solve(n, 5, 5, h, B, nroots=1, e_core=e0, tol=1e-12)
    rh, rB, rE = _oracle(h, B, C[0], space, e0)
    ref = json.load(open(GOLDEN))["cas10_nq48_s0"]["energies"][0]
    print(f"E_dmrg-E_fci={eg[0] - ref:.2e} |ddh|={np.abs(dh - rh).max():.2e} |ddB|={np.abs(dB - rB).max():.2e}")
    assert abs(eg[0] - ref) <= 1e-10
    assert np.abs(dh - rh).max() <= 1e-10
    assert np.abs(dB - rB).max() <= 1e-10


def test_grad_state_averaged_roots_cas6():
    """Per-root and weighted gradients of a 3-root state-averaged run at full bond."""
    pk = _pk()
    n, nq = 6, 12
    h, B, e0 = synth.make_hamiltonian(n, nq, 3)
    sol = pk.Solver(pk.Problem(h, B, 3, 3, e0), M=64, n_states=3, tol=1e-12)
    sol.sweep(3)
    E, C, space = fci.solve(n, 3, 3, h, B, nroots=3, e_core=e0)
    per = []
    for r in range(3):
        w = np.zeros(3)
        w[r] = 1.0
        dh, dB, eg = sol.grad(w)
        rh, rB, rE = _oracle(h, B, C[r], space, e0)
        assert abs(eg[r] - E[r]) <= 1e-10
        assert np.abs(dh - rh).max() <= 1e-9
        assert np.abs(dB - rB).max() <= 1e-9
        per.append((dh, dB))
    w = np.array([0.5, 0.3, 0.2])
    dh, dB, _ = sol.grad(w)
    assert np.abs(dh - sum(w[r] * per[r][0] for r in range(3))).max() <= 1e-12
    assert np.abs(dB - sum(w[r] * per[r][1] for r in range(3))).max() <= 1e-12


def test_grad_matches_central_finite_difference_cas6():
    """d/de E(h + e dh, B + e dB) by the five-point central difference of
    full-bond DMRG runs (truncation error O(eps^4), noise ~1e-13 / eps)."""
    pk = _pk()
    n, nq, eps = 6, 12, 1e-4
    h, B, e0 = synth.make_hamiltonian(n, nq, 0)
    rng = np.random.default_rng(42)
    Dh = rng.normal(size=(n, n))
    Dh = Dh + Dh.T
    DB = rng.normal(size=(nq, n, n))
    DB = DB + DB.transpose(0, 2, 1)

    def energy(hh, BB):
        s = pk.Solver(pk.Problem(hh, BB, 3, 3, e0), M=64, tol=1e-12)
        s.sweep(2)
        return s.energy()[0], s

    _, sol = energy(h, B)
    dh, dB, _ = sol.grad()
    analytic = np.sum(dh * Dh) + np.sum(dB * DB)
    f = {t: energy(h + t * eps * Dh, B + t * eps * DB)[0] for t in (-2, -1, 1, 2)}
    fd = (f[-2] - 8 * f[-1] + 8 * f[1] - f[2]) / (12 * eps)
    print(f"analytic={analytic:.12f} fd={fd:.12f} diff={analytic - fd:.2e}")
    assert abs(analytic - fd) <= 1e-7 * max(1.0, abs(analytic))


def test_grad_invariants_cas12_m256():
    """Truncated bond, larger active space: properties that hold for any state.
    trace(dE/dh) = N_el, dE/dh symmetric, and Euler's identity
    sum h dE/dh + 1/2 sum B dE/dB = E - e_core (E is of degree 1 in h and 2 in B)."""
    pk = _pk()
    n, nq = 12, 64
    h, B, e0 = synth.make_hamiltonian(n, nq, 0)
    e0 = -1.5
    sol = pk.Solver(pk.Problem(h, B, 6, 6, e0), M=256, tol=1e-9)
    sol.sweep(1)
    dh, dB, eg = sol.grad()
    assert abs(np.trace(dh) - 12.0) <= 1e-10
    assert np.abs(dh - dh.T).max() <= 1e-10
    euler = np.sum(h * dh) + 0.5 * np.sum(B * dB)
    assert abs(euler - (eg[0] - e0)) <= 1e-9 * max(1.0, abs(euler))
    assert abs(eg[0] - sol.energy()[0]) <= 1e-9


def test_autograd_function_backward_is_dmrg_grad():
    import torch
    pk = _pk()
    n, nq = 4, 6
    h, B, e0 = synth.make_hamiltonian(n, nq, 1)
    ht = torch.tensor(h, requires_grad=True)
    Bt = torch.tensor(B, requires_grad=True)
    e = pk.dmrg_energy(ht, Bt, 2, 2, e0, n_sweeps=3, M=64, n_states=2, tol=1e-12)
    assert e.shape == (2,)
    (2.0 * e[0] - 0.5 * e[1]).backward()
    E, C, space = fci.solve(n, 2, 2, h, B, nroots=2, e_core=e0)
    g = [_oracle(h, B, C[r], space, e0) for r in range(2)]
    assert np.abs(e.detach().numpy() - E).max() <= 1e-10
    assert np.abs(ht.grad.numpy() - (2.0 * g[0][0] - 0.5 * g[1][0])).max() <= 1e-9
    assert np.abs(Bt.grad.numpy() - (2.0 * g[0][1] - 0.5 * g[1][1])).max() <= 1e-9


def test_config4_two_roots_cas16_m512_finite_difference_gap():
    """Configuration 4: CAS(16,16), N_Q = 96, M = 512 (truncated: the full middle
    bond is 65536), 2 state-averaged roots.  Per-root gradients of the final MPS
    against the central finite difference (step 1e-5) of each root's sweep
    energy along a random symmetric direction, each side a full DMRG run from the
    same start.  At truncated bond the fixed-MPS gradient is not the derivative
    of the sweep energy (the sweep re-optimises a truncated state; Sec. II.E):
    the gap is reported beside tau and checked only for its size."""
    pk = _pk()
    n, nq, Mb, eps = 16, 96, 512, 1e-5
    h, B, e0 = synth.make_hamiltonian(n, nq, 0)
    rng = np.random.default_rng(7)
    Dh = rng.normal(size=(n, n))
    Dh = Dh + Dh.T
    DB = rng.normal(size=(nq, n, n))
    DB = DB + DB.transpose(0, 2, 1)

    def run(hh, BB):
        s = pk.Solver(pk.Problem(hh, BB, n // 2, n // 2, e0), M=Mb, n_states=2, tol=1e-9)
        e, tau, ok = s.sweep(4)
        return s, s.energy(), tau, ok

    sol, e, tau, ok = run(h, B)
    ep = run(h + eps * Dh, B + eps * DB)[1]
    em = run(h - eps * Dh, B - eps * DB)[1]
    assert ok
    for r in range(2):
        w = np.zeros(2)
        w[r] = 1.0
        dh, dB, er = sol.grad(w)
        analytic = float(np.sum(dh * Dh) + np.sum(dB * DB))
        fd = float((ep[r] - em[r]) / (2 * eps))
        gap = abs(analytic - fd)
        print(f"root {r}: E={e[r]:.10f} analytic={analytic:.9f} fd={fd:.9f} gap={gap:.3e} "
              f"(relative {gap / abs(analytic):.1e}) tau={tau:.2e}", flush=True)
        assert abs(np.trace(dh) - n) <= 1e-9  # the gradient of a normalised N-electron state
        assert abs(er[r] - e[r]) <= 1e-9
        # the gap tracks the truncation, not a mistake: small against the derivative itself
        assert gap <= 1e-3 * abs(analytic)
    # the state-averaged energy is the one the sweep makes stationary: its
    # gradient (the weighted sum of the roots') matches its finite difference
    # far more closely than a single root's
    dh, dB, _ = sol.grad(np.array([0.5, 0.5]))
    analytic = float(np.sum(dh * Dh) + np.sum(dB * DB))
    fd = float((0.5 * (ep[0] + ep[1]) - 0.5 * (em[0] + em[1])) / (2 * eps))
    print(f"state average: analytic={analytic:.9f} fd={fd:.9f} gap={abs(analytic - fd):.3e}", flush=True)
    assert abs(analytic - fd) <= 1e-6 * abs(analytic)


def _stationary(sol, max_sweeps=200, tol=1e-7):
    """One-site sweeps until the largest local tangent gradient is below tol."""
    for _ in range(max_sweeps):
        e, res, ok = sol.stationarize(1)
        if res <= tol:
            return e, res
    return e, res


def test_stationary_truncated_mps_gradient_equals_finite_difference():
    """CAS(8,8), N_Q = 32 at M = 24 (truncated, tau ~ 1e-2).  The two-site fixed point is
    not tangent-stationary: its Hellmann-Feynman gradient misses the central
    finite difference of the two-site DMRG energy by an amount of the order of
    the discarded weight.  One-site sweeps at the same bond dimensions drive the
    gauge-free tangent gradient to zero (1e-7: one-site sweeps converge
    linearly); then dmrg_grad equals the central finite difference (step 1e-4
    along a random symmetric h direction) of the stationary energy at that bond
    dimension to 1e-5, and the energy is variational."""
    pk = _pk()
    h, B, e0 = synth.make_hamiltonian(8, 32, 0)
    e_fci = json.load(open(GOLDEN))["cas8_nq32_s0"]["energies"][0]
    M, eps = 24, 1e-4
    rng = np.random.default_rng(5)
    D = rng.normal(size=(8, 8))
    D = D + D.T
    sol = pk.Solver(pk.Problem(h, B, 4, 4, e0), M=M, tol=1e-11)
    e2, tau, _ = sol.sweep(6)
    dh2, _, _ = sol.grad()
    two = sol.export_mps()
    e_two_state = sol.energy()[0]
    es, res = _stationary(sol)
    assert res <= 1e-7, res
    dh, _, (e_grad,) = sol.grad()
    stat = sol.export_mps()

    def energy(sign, start, stationary):
        s = pk.Solver(pk.Problem(h + sign * eps * D, B, 4, 4, e0), M=M, tol=1e-11)
        s.set_mps(start["bonds"], start["sites"])
        if stationary:
            s.sweep(1)  # canonical form with the centre on site 0 (nothing to truncate at these bonds)
            return _stationary(s)[0]
        return s.sweep(6)[0][0]

    fd = (energy(1, stat, True) - energy(-1, stat, True)) / (2 * eps)
    fd2 = (energy(1, two, False) - energy(-1, two, False)) / (2 * eps)
    hf, hf2 = float(np.sum(dh * D)), float(np.sum(dh2 * D))
    print(f"tau {tau:.2e}; two-site: E(Ritz) {e2[0]:.10f} E(state) {e_two_state:.10f} FD {fd2:.8f} HF {hf2:.8f} "
          f"gap {abs(fd2 - hf2):.2e}; stationary: E {es:.10f} res {res:.1e} FD {fd:.8f} HF {hf:.8f} "
          f"gap {abs(fd - hf):.2e}", flush=True)
    assert abs(e_grad - es) <= 1e-10
    assert e_fci - 1e-10 <= es <= e_two_state + 1e-10
    assert abs(fd - hf) <= 1e-5 * max(1.0, abs(hf))
