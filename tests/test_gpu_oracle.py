"""GPU parity against the block-sparse oracle (oracle.mpo / oracle.blocks /
oracle.truncate: its own MPO and environments, sharing no code with the HIP
path), through the C ABI: the H_eff diagonal, sigma at the benched workload
(CAS(20,20), N_Q = 120, M = 1024, middle bond) on the GPU's own MPS, the SVD
truncation, and MPS energies at truncated bond against FCI bounds."""
import json
import os
import time

import numpy as np
import pytest

import synth
from oracle import blocks, embed, truncate
from oracle import mpo as om

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fci_energies.json")


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _gold(name):
    return json.load(open(GOLD))[name]


@pytest.mark.parametrize("n,na,nb,nq,M,k", [(4, 2, 2, 5, 16, 1), (6, 3, 3, 8, 12, 0), (6, 3, 2, 8, 20, 4),
                                            (8, 4, 4, 16, 40, 3), (10, 5, 5, 12, 200, 4)])
def test_diag_matches_oracle(n, na, nb, nq, M, k):
    torch = _torch()
    import paper_2609_09990_amd as pk
    print(f"diag case n={n} M={M} k={k}", flush=True)
    h, B, e0 = synth.make_hamiltonian(n, nq, 2)
    sol = pk.Solver(pk.Problem(h, B, na, nb, e0), M=M)
    mps = synth.random_mps(n, na, nb, M, seed=8)
    sol.set_mps(mps["bonds"], mps["sites"])
    size = sol.prepare(k)
    d = torch.zeros(size, dtype=torch.float64, device="cuda")
    sol.diag(k, d)
    ref = blocks.TwoSite(om.build_mpo(h, B), mps, k).diag()
    got = d.cpu().numpy()
    assert np.max(np.abs(got - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_sigma_and_diag_sampled_blocks_vs_oracle_cas20_m1024():
    """The benched configuration: CAS(20,20), N_Q = 120, M = 1024, FP64, step k = 9
    after a left-to-right half sweep from the solver's seeded start (the launch
    configuration bench.py times).  The MPS is the GPU's own (dmrg_export_mps:
    data, not code); the oracle builds its own MPO and environments from it and
    computes sampled output blocks of sigma and of the diagonal one by one."""
    torch = _torch()
    import paper_2609_09990_amd as pk
    h, B, e0 = synth.make_hamiltonian(20, 120, 0)
    sol = pk.Solver(pk.Problem(h, B, 10, 10, e0), M=1024, tol=1e-8)
    t0 = time.time()
    for k in range(9):
        sol.step(k, 0)
    k = 9
    n = sol.prepare(k)
    mps = sol.export_mps()
    print(f"GPU half sweep {time.time() - t0:.1f} s, |psi| = {n}, bond {k + 1} = "
          f"{sum(d for *_, d in mps['bonds'][k + 1])}", flush=True)
    psi = np.random.default_rng(17).standard_normal(n)
    psi /= np.linalg.norm(psi)
    x = torch.from_numpy(psi).cuda()
    y = torch.zeros_like(x)
    d = torch.zeros_like(x)
    sol.sigma(k, x, y)
    sol.diag(k, d)
    torch.cuda.synchronize()
    sig = y.cpu().numpy()
    dia = d.cpu().numpy()
    t1 = time.time()
    ts = blocks.TwoSite(om.build_mpo(h, B), mps, k, progress=lambda m: print("oracle:", m, flush=True))
    print(f"oracle environments {time.time() - t1:.1f} s", flush=True)
    out = ts.output_blocks()
    size = {key: ts.bl.dim(key[0]) * ts.br.dim(key[2]) for key in out}
    rng = np.random.default_rng(5)
    largest = sorted(out, key=lambda key: -size[key])[:6]
    smallest = sorted(out, key=lambda key: size[key])[:4]
    rand = [out[i] for i in rng.choice(len(out), 10, replace=False)]
    pick = list(dict.fromkeys(largest + smallest + rand))
    t2 = time.time()
    ref = ts.sigma(psi, blocks=pick)
    refd = ts.diag(blocks=pick)
    print(f"oracle {len(pick)} sampled blocks {time.time() - t2:.1f} s", flush=True)
    got = blocks.unpack(ts.bl, ts.br, blocks.twosite_qn(), sig)
    gotd = blocks.unpack(ts.bl, ts.br, blocks.twosite_qn(), dia)
    num = sum(np.sum((got[key] - ref[key]) ** 2) for key in pick)
    den = sum(np.sum(ref[key] ** 2) for key in pick)
    err = np.sqrt(num / den)
    dmax = max(np.max(np.abs(gotd[key] - refd[key])) for key in pick)
    dref = max(np.max(np.abs(refd[key])) for key in pick)
    print(f"sampled sigma norm-relative error {err:.2e} over {len(pick)} blocks "
          f"({sum(size[key] for key in pick)} elements), diag max error {dmax:.2e}", flush=True)
    assert err <= 1e-12
    assert dmax <= 1e-12 * dref


def _constructed(bonds, k, seed):
    """Sector spectra (normalised: sum s^2 = 1) with one exactly degenerate
    mirror pair (N, +2Sz) / (N, -2Sz) at a value v near the median; returns
    (spectra, v)."""
    bk, bk2 = blocks.Bond(bonds[k]), blocks.Bond(bonds[k + 2])
    size = {}
    for qm, rows, cols in truncate.middle_sectors(bk, bk2):
        size[qm] = min(sum(bk.dim(a) for _, a in rows), sum(bk2.dim(b) for _, b in cols))
    rng = np.random.default_rng(seed)
    spectra = {qm: np.sort(rng.uniform(0.05, 1.0, s))[::-1] for qm, s in size.items()}
    pair = next(q for q in size if q[1] > 0 and size[q] >= 2 and size.get((q[0], -q[1]), 0) >= 2)
    mirror = (pair[0], -pair[1])
    v = float(np.median(np.concatenate(list(spectra.values()))))
    spectra[pair] = np.sort(np.append(spectra[pair][:-1], v))[::-1]
    spectra[mirror] = np.sort(np.append(spectra[mirror][:-1], v))[::-1]
    tot = np.sqrt(sum(np.sum(s ** 2) for s in spectra.values()))
    return {q: s / tot for q, s in spectra.items()}, v / tot


@pytest.mark.parametrize("direction,n_states", [(0, 1), (1, 1), (0, 2), (1, 2)])
def test_truncation_matches_oracle(direction, n_states):
    """dmrg_truncate on given two-site vectors against the oracle's per-sector
    SVD: new bond sectors, tau, and the kept singular values (their squares to
    1e-13: the HIP path takes them from density-matrix eigenvalues).  For one
    root the spectrum has an exactly degenerate mirror pair at the cut, which
    the cluster rule must keep or drop together."""
    torch = _torch()
    import paper_2609_09990_amd as pk
    n, na, nb, k = 8, 4, 4, 3
    h, B, e0 = synth.make_hamiltonian(n, 16, 4)
    mps = synth.random_mps(n, na, nb, 64, seed=9)
    bonds = mps["bonds"]
    w = [0.6, 0.4][:n_states]
    if n_states == 1:
        spectra, v = _constructed(bonds, k, 3)
        psis = [truncate.psi_from_spectra(bonds[k], bonds[k + 2], spectra, seed=4)]
        vals = np.sort(np.concatenate(list(spectra.values())))[::-1]
        i = int(np.nonzero(np.abs(vals - v) <= 1e-15)[0][0])
        Mcut = i + 1  # the cut falls between the two copies of v
    else:
        psis = [synth.random_twosite(bonds, k, seed=20 + r) for r in range(n_states)]
        full = len(truncate.truncate(psis, bonds[k], bonds[k + 2], 10 ** 6, weights=w)["kept"])
        Mcut = full // 2
    ref = truncate.truncate(psis, bonds[k], bonds[k + 2], Mcut, left_to_right=(direction == 0),
                            weights=w if n_states > 1 else None)
    sol = pk.Solver(pk.Problem(h, B, na, nb, e0), M=Mcut, n_states=n_states,
                    weights=w if n_states > 1 else None)
    sol.set_mps(bonds, mps["sites"])
    x = torch.from_numpy(np.concatenate(psis)).cuda()
    tau, sv = sol.truncate(k, x, direction)
    newbond = [tuple(s) for s in sol.bonds()[k + 1]]
    print(f"dir={direction} roots={n_states} M={Mcut}: kept {len(sv)} (oracle {len(ref['kept'])}), "
          f"tau {tau:.3e} (oracle {ref['tau']:.3e})", flush=True)
    assert newbond == [tuple(s) for s in ref["bond"]]
    assert len(sv) == len(ref["kept"])
    assert np.max(np.abs(sv ** 2 - ref["kept"] ** 2)) <= 1e-13
    assert abs(tau - ref["tau"]) <= 1e-13
    if n_states == 1:
        assert len(sv) < Mcut  # the cut moved up to keep the degenerate pair together


def test_truncated_sweep_energy_vs_oracle_cas8_m64():
    """CAS(8,8), N_Q = 32 at M = 64 (the full middle bond is 256): the GPU's MPS
    expectation energy equals the oracle's <Psi|H|Psi>/<Psi|Psi> of the exported
    MPS (determinant space), and it lies above FCI (variational bound)."""
    torch = _torch()
    import paper_2609_09990_amd as pk
    h, B, e0 = synth.make_hamiltonian(8, 32, 0)
    sol = pk.Solver(pk.Problem(h, B, 4, 4, e0), M=64, tol=1e-10)
    e, tau, ok = sol.sweep(3)
    em = sol.energy()[0]
    mps = sol.export_mps()
    ref = embed.mps_energy(h, B, mps, 4, 4, e0)
    efci = _gold("cas8_nq32_s0")["energies"][0]
    print(f"CAS(8,8) M=64: E_mps {em:.12f} oracle {ref:.12f} E-E_fci {em - efci:.3e} tau {tau:.2e}", flush=True)
    assert ok
    assert tau > 0  # the bond really is truncated
    assert abs(em - ref) <= 1e-10
    assert em >= efci - 1e-12


def _energy_from_centre(h, B, mps, nq_mpo=None):
    """<Psi|H|Psi>/<Psi|Psi> from the two-site tensor at sites (0, 1) of an MPS
    whose sites 2.. are right-orthonormal (the oracle's own H_eff at k = 0)."""
    assert blocks.right_orthonormality_error(mps, 2) < 1e-10
    ts = blocks.TwoSite(om.build_mpo(h, B), mps, 0)
    psi = blocks.twosite_from_sites(mps, 0)
    return float(psi @ ts.sigma(psi) / (psi @ psi))


def test_config2_state_averaged_cas12_m512_bounds():
    """CAS(12,12), N_Q = 64, 3 lowest roots state-averaged at M = 512 (truncated:
    the full middle bond is 4096).  Against FCI: every Ritz value lies above its
    FCI eigenvalue (Cauchy interlacing) and the MPS energy of root 0 equals the
    oracle's energy of the exported MPS; E - E_FCI and tau are reported per root."""
    torch = _torch()
    import paper_2609_09990_amd as pk
    h, B, e0 = synth.make_hamiltonian(12, 64, 0)
    g = _gold("cas12_nq64_s0")["energies"]
    sol = pk.Solver(pk.Problem(h, B, 6, 6, e0), M=512, n_states=3, tol=1e-9)
    t0 = time.time()
    e, tau, ok = sol.sweep(3)
    em = sol.energy()
    mps = sol.export_mps()
    ref0 = _energy_from_centre(h, B, mps)
    print(f"CAS(12,12) SA-3 M=512 ({time.time() - t0:.1f} s): Ritz {e}, MPS {em}, "
          f"E-E_fci {np.array(e) - np.array(g)}, tau {tau:.2e}, oracle root0 {ref0:.12f}", flush=True)
    assert ok
    for r in range(3):
        assert e[r] >= g[r] - 1e-10
        assert em[r] >= g[r] - 1e-10
    assert abs(em[0] - ref0) <= 1e-10


def test_config2_exact_bond_cas12_equals_fci():
    """CAS(12,12), N_Q = 64, 3 roots at M = 4096 (the full middle bond): DMRG = FCI
    to 1e-10 for every root."""
    torch = _torch()
    import paper_2609_09990_amd as pk
    h, B, e0 = synth.make_hamiltonian(12, 64, 0)
    g = _gold("cas12_nq64_s0")["energies"]
    sol = pk.Solver(pk.Problem(h, B, 6, 6, e0), M=4096, n_states=3, tol=1e-10)
    t0 = time.time()
    e, tau, ok = sol.sweep(2)
    print(f"CAS(12,12) SA-3 M=4096 ({time.time() - t0:.1f} s): E-E_fci {np.array(e) - np.array(g)}, tau {tau:.2e}, "
          f"matvecs {sol.stats()['matvecs']:.0f}", flush=True)
    assert ok
    assert np.max(np.abs(np.array(e) - np.array(g))) <= 1e-10


@pytest.mark.parametrize("direction", [0, 1])
def test_adaptive_truncation_matches_oracle(direction):
    """trunc_tol (adaptive bond dimension) on a constructed spectrum with a
    degenerate mirror pair: the tolerance falls where it would keep one copy of
    the pair, so the cut keeps both; new bond, tau and kept values as the oracle."""
    torch = _torch()
    import paper_2609_09990_amd as pk
    n, na, nb, k = 8, 4, 4, 3
    h, B, e0 = synth.make_hamiltonian(n, 16, 4)
    mps = synth.random_mps(n, na, nb, 64, seed=9)
    bonds = mps["bonds"]
    spectra, v = _constructed(bonds, k, 3)
    psis = [truncate.psi_from_spectra(bonds[k], bonds[k + 2], spectra, seed=4)]
    vals = np.sort(np.concatenate(list(spectra.values())))[::-1]
    i = int(np.nonzero(np.abs(vals - v) <= 1e-15)[0][0])  # first copy of v
    w = vals ** 2
    tol = float(np.sum(w[i + 1:]) + 0.5 * w[i])  # room for dropping one copy of v, not two
    ref = truncate.truncate(psis, bonds[k], bonds[k + 2], 4096, left_to_right=(direction == 0), trunc_tol=tol)
    sol = pk.Solver(pk.Problem(h, B, na, nb, e0), M=4096, trunc_tol=tol)
    sol.set_mps(bonds, mps["sites"])
    tau, sv = sol.truncate(k, torch.from_numpy(np.concatenate(psis)).cuda(), direction)
    newbond = [tuple(s) for s in sol.bonds()[k + 1]]
    print(f"dir={direction}: kept {len(sv)} (oracle {len(ref['kept'])}, first copy at {i}), tau {tau:.3e} "
          f"(oracle {ref['tau']:.3e}, tol {tol:.3e})", flush=True)
    assert len(ref["kept"]) == i + 2  # both copies kept
    assert newbond == [tuple(s) for s in ref["bond"]]
    assert len(sv) == len(ref["kept"])
    assert np.max(np.abs(sv ** 2 - ref["kept"] ** 2)) <= 1e-13
    assert abs(tau - ref["tau"]) <= 1e-13 and tau <= tol


def test_adaptive_bond_dimension_dmrg_cas8():
    """CAS(8,8), N_Q = 32 with trunc_tol = 1e-6 and M = 4096: the bond
    dimensions adapt per bond (below the full bonds, not all equal), every
    truncation of the last sweep discards at most the tolerance, and the energy
    lies above the oracle's FCI energy by less than 1e-4 Ha."""
    _torch()
    import paper_2609_09990_amd as pk
    gold = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fci_energies.json")))
    e_fci = gold["cas8_nq32_s0"]["energies"][0]
    h, B, e0 = synth.make_hamiltonian(8, 32, 0)
    sol = pk.Solver(pk.Problem(h, B, 4, 4, e0), M=4096, tol=1e-9, trunc_tol=1e-6)
    for _ in range(4):
        e, tau, ok = sol.sweep(1)
    dims = [sum(d for _, _, d in b) for b in sol.bonds()]
    full = [sum(d for _, _, d in b) for b in synth.random_mps(8, 4, 4, 10 ** 6, seed=0)["bonds"]]
    print(f"E {e[0]:.10f} FCI {e_fci:.10f} dE {e[0] - e_fci:.2e} tau {tau:.2e} bonds {dims} full {full}", flush=True)
    assert tau <= 1e-6
    assert -1e-9 <= e[0] - e_fci <= 1e-4
    assert all(d <= f for d, f in zip(dims, full)) and sum(dims) < sum(full)
    assert len(set(dims[2:-2])) > 1
