"""GPU parity of the HIP sigma path against the CPU oracle (through the C ABI)."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import embed

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fci_energies.json")


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _setup(n, na, nb, nq, M, seed_h=0, seed_mps=5):
    torch = _torch()
    import paper_2609_09990_amd as pk
    h, B, e0 = synth.make_hamiltonian(n, nq, seed_h)
    prob = pk.Problem(h, B, na, nb, e0)
    sol = pk.Solver(prob, M=M)
    mps = synth.random_mps(n, na, nb, M, seed=seed_mps)
    sol.set_mps(mps["bonds"], mps["sites"])
    return torch, pk, h, B, prob, sol, mps


@pytest.mark.parametrize("n,na,nb,nq,M,k", [
    (4, 2, 2, 5, 16, 1),       # tiny, full bonds
    (6, 3, 3, 8, 12, 0),       # left edge, truncated (ragged) sectors
    (6, 3, 3, 8, 12, 2),
    (6, 3, 2, 8, 20, 4),       # right edge, odd electron count
    (8, 4, 4, 16, 40, 3),
    (10, 5, 5, 12, 1024, 4),   # middle of CAS(10,10) at full bond: blocks of 100 (two tiles + tail)
])
def test_sigma_matches_oracle_projection(n, na, nb, nq, M, k):
    torch, pk, h, B, prob, sol, mps = _setup(n, na, nb, nq, M)
    print(f"case n={n} M={M} k={k}", flush=True)
    size = sol.prepare(k)
    psi = synth.random_twosite(mps["bonds"], k, seed=11)
    assert psi.size == size
    ref = embed.sigma_twosite(h, B, mps, k, psi, na, nb)
    d_psi = torch.from_numpy(psi).cuda()
    d_out = torch.zeros_like(d_psi)
    flops = sol.sigma(k, d_psi, d_out)
    torch.cuda.synchronize()
    got = d_out.cpu().numpy()
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err <= 1e-12, err
    assert flops > 0


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 2e-6)])
def test_chunked_sigma_matches_oracle(prec, tol):
    """Sigma intermediates bounded to 1 MiB (many chunks of left factors, phase B
    adding into sigma chunk by chunk) at CAS(10,10), M = 1024, middle bond: the
    same sigma as the oracle, in fp64 and in fp32."""
    torch = _torch()
    import paper_2609_09990_amd as pk
    h, B, e0 = synth.make_hamiltonian(10, 12, 0)
    prob = pk.Problem(h, B, 5, 5, e0)
    mps = synth.random_mps(10, 5, 5, 1024, seed=5)
    k = 4
    psi = synth.random_twosite(mps["bonds"], k, seed=11)
    ref = embed.sigma_twosite(h, B, mps, k, psi, 5, 5)
    outs = []
    for chunk in (0, 1 << 20):
        sol = pk.Solver(prob, M=1024, sigma_chunk_bytes=chunk)
        sol.set_mps(mps["bonds"], mps["sites"])
        sol.prepare(k)
        d_psi = torch.from_numpy(psi).cuda()
        d_out = torch.zeros_like(d_psi)
        sol.sigma(k, d_psi, d_out, prec)
        torch.cuda.synchronize()
        outs.append(d_out.cpu().numpy())
        err = np.linalg.norm(outs[-1] - ref) / np.linalg.norm(ref)
        print(f"chunk={chunk} prec={prec} err={err:.2e}", flush=True)
        assert err <= tol, err
    assert np.linalg.norm(outs[0] - outs[1]) <= 4 * tol * np.linalg.norm(ref)


def test_sigma_hermitian_and_deterministic():
    torch, pk, h, B, prob, sol, mps = _setup(8, 4, 4, 16, 60)
    k = 3
    size = sol.prepare(k)
    rng = np.random.default_rng(3)
    x = torch.from_numpy(rng.standard_normal(size)).cuda()
    y = torch.from_numpy(rng.standard_normal(size)).cuda()
    hx, hy, hx2 = torch.zeros_like(x), torch.zeros_like(x), torch.zeros_like(x)
    sol.sigma(k, x, hx)
    sol.sigma(k, y, hy)
    sol.sigma(k, x, hx2)
    torch.cuda.synchronize()
    a = float(torch.dot(x, hy))
    b = float(torch.dot(y, hx))
    assert abs(a - b) <= 1e-12 * float(torch.norm(hx)) * float(torch.norm(y))
    assert torch.equal(hx, hx2)  # fixed summation order: bitwise reproducible


def test_diag_matches_sigma_on_unit_vectors():
    torch, pk, h, B, prob, sol, mps = _setup(6, 3, 3, 8, 30)
    k = 2
    size = sol.prepare(k)
    d = torch.zeros(size, dtype=torch.float64, device="cuda")
    sol.diag(k, d)
    rng = np.random.default_rng(0)
    idx = rng.choice(size, size=min(size, 25), replace=False)
    for i in idx:
        e = torch.zeros(size, dtype=torch.float64, device="cuda")
        e[int(i)] = 1.0
        out = torch.zeros_like(e)
        sol.sigma(k, e, out)
        torch.cuda.synchronize()
        assert abs(float(out[int(i)]) - float(d[int(i)])) <= 1e-12 * max(1.0, abs(float(d[int(i)])))


# Rounding the operands once (fp32 unit roundoff 6e-8, bf16 3.9e-3) with fp32
# accumulation gives relative errors of a few units of the operand roundoff
# here (2e-7 and 4e-3 with exact rounding on the CPU).
@pytest.mark.parametrize("prec,tol", [(1, 2e-6), (2, 1e-2)])
def test_low_precision_sigma_close_to_fp64(prec, tol):
    torch, pk, h, B, prob, sol, mps = _setup(8, 4, 4, 16, 60)
    k = 3
    size = sol.prepare(k)
    psi = torch.from_numpy(synth.random_twosite(mps["bonds"], k, seed=4)).cuda()
    o64, olo = torch.zeros_like(psi), torch.zeros_like(psi)
    sol.sigma(k, psi, o64, 0)
    sol.sigma(k, psi, olo, prec)
    torch.cuda.synchronize()
    err = float(torch.norm(olo - o64) / torch.norm(o64))
    assert err < tol, err


@pytest.mark.parametrize("prec,tol", [(1, 2e-6), (2, 1e-2)])
def test_shifted_low_precision_sigma_at_the_centre(prec, tol):
    """With the orthogonality centre on the two sites the low-precision copies
    hold the block Hamiltonians shifted by their diagonal means and the product
    adds the shift back in fp64: the result is the same sigma as fp64, to the
    low precision's tolerance, and no farther from it than without the shift."""
    torch = _torch()
    import paper_2609_09990_amd as pk
    h, B, e0 = synth.make_hamiltonian(10, 12, 0)
    prob = pk.Problem(h, B, 5, 5, e0)
    sol = pk.Solver(prob, M=200, tol=1e-6)
    for k in range(4):
        sol.step(k, 0)
    k = 4  # centre on site 4 after the steps
    mps = sol.export_mps()
    plain = pk.Solver(prob, M=200)
    plain.set_mps(mps["bonds"], mps["sites"])  # gauge unknown: no shift
    errs = []
    for s in (sol, plain):
        n = s.prepare(k)
        x = torch.from_numpy(synth.random_twosite(mps["bonds"], k, seed=9)).cuda()
        y64, ylo = torch.zeros_like(x), torch.zeros_like(x)
        s.sigma(k, x, y64, 0)
        s.sigma(k, x, ylo, prec)
        torch.cuda.synchronize()
        errs.append(float(torch.norm(ylo - y64) / torch.norm(y64)))
    print(f"prec={prec}: shifted {errs[0]:.2e}, plain {errs[1]:.2e}", flush=True)
    assert errs[0] < tol
    assert errs[0] <= 1.5 * errs[1]


def _gold(name):
    return json.load(open(GOLD))[name]


def test_dmrg_full_bond_equals_fci_cas8():
    """CAS(8,8), 32 Cholesky vectors, M = 256 = full middle bond: DMRG = FCI."""
    torch = _torch()
    import paper_2609_09990_amd as pk
    g = _gold("cas8_nq32_s0")
    h, B, e0 = synth.make_hamiltonian(8, 32, 0)
    prob = pk.Problem(h, B, 4, 4, e0)
    sol = pk.Solver(prob, M=256, tol=1e-10)
    e, tau, ok = sol.sweep(4)
    em = sol.energy()
    print("cas8 E", e, "mps", em, "fci", g["energies"][0], "tau", tau, sol.stats(), flush=True)
    assert ok
    assert abs(e[0] - g["energies"][0]) <= 1e-10
    assert abs(em[0] - g["energies"][0]) <= 1e-10


def test_state_averaged_full_bond_cas6():
    torch = _torch()
    import paper_2609_09990_amd as pk
    g = _gold("cas6_nq12_s3")
    h, B, e0 = synth.make_hamiltonian(6, 12, 3)
    prob = pk.Problem(h, B, 3, 3, e0)
    sol = pk.Solver(prob, M=64, n_states=3, tol=1e-10)
    e, tau, ok = sol.sweep(3)
    print("cas6 SA", e, g["energies"], flush=True)
    assert ok
    assert np.max(np.abs(np.array(e) - np.array(g["energies"]))) <= 1e-10


@pytest.mark.parametrize("prec", [1, 2])
def test_precision_form_full_bond_equals_fci_cas8(prec):
    """FP32 / BF16 sigma with the switch to fp64 (defect correction): every step
    converges on an fp64 residual, so at full bond the energy is FCI's."""
    _torch()
    import paper_2609_09990_amd as pk
    h, B, e0 = synth.make_hamiltonian(8, 32, 0)
    sol = pk.Solver(pk.Problem(h, B, 4, 4, e0), M=256, tol=1e-10, precision=prec)
    e, tau, ok = sol.sweep(2)
    ref = json.load(open(GOLD))["cas8_nq32_s0"]["energies"][0]
    st = sol.stats()
    print(f"prec={prec} E-E_fci={e[0] - ref:.2e} matvecs={st['matvecs']:.0f} switches={st['refinements']:.0f}")
    assert ok
    assert abs(e[0] - ref) <= 1e-10
    assert abs(sol.energy()[0] - ref) <= 1e-10
    assert st["refinements"] > 0
    assert st["lowp_matvecs"] > 0  # the low-precision kernels really ran


def test_executed_flops_at_most_algorithmic():
    """The merged / trimmed plan executes no more block-product flops than the
    factorisation's algorithmic count, and the sigma it computes is unchanged
    (parity above); the two counts are reported separately."""
    _torch()
    import paper_2609_09990_amd as pk
    h, B, e0 = synth.make_hamiltonian(8, 32, 0)
    sol = pk.Solver(pk.Problem(h, B, 4, 4, e0), M=64, tol=1e-9)
    sol.sweep(1)
    st = sol.stats()
    assert 0 < st["sigma_a_flops_exec"] <= st["sigma_a_flops"]
    assert 0 < st["sigma_b_flops_exec"] <= st["sigma_b_flops"]
    assert abs(st["sigma_flops"] - st["sigma_a_flops"] - st["sigma_b_flops"]) <= 1e-6 * st["sigma_flops"]


def test_cached_step_plan_gives_the_same_sigma():
    """A revisited step reuses its cached plan (factor premix and merged right
    blocks rerun against the current environments): the sigma is bitwise equal
    to the one computed from the freshly built plan, and equal to the oracle's."""
    torch, pk, h, B, prob, sol, mps = _setup(8, 4, 4, 16, 40)
    k = 3
    size = sol.prepare(k)
    psi = synth.random_twosite(mps["bonds"], k, seed=21)
    x = torch.from_numpy(psi).cuda()
    y1, y2 = torch.zeros_like(x), torch.zeros_like(x)
    sol.sigma(k, x, y1)
    hits0 = sol.stats()["plan_hits"]
    sol.prepare(k + 1)
    assert sol.prepare(k) == size
    sol.sigma(k, x, y2)
    torch.cuda.synchronize()
    assert sol.stats()["plan_hits"] == hits0 + 1
    assert torch.equal(y1, y2)
    ref = embed.sigma_twosite(h, B, mps, k, psi, 4, 4)
    err = np.linalg.norm(y2.cpu().numpy() - ref) / np.linalg.norm(ref)
    assert err <= 1e-12, err


def test_full_size_sigma_properties_cas20_m1024():
    """The bench workload (CAS(20,20), N_Q = 120, M = 1024, middle bond, the
    launch configuration bench.py times): no oracle reaches this size, so the
    checks are properties that hold at any size: the step converges, H_eff is
    symmetric, sigma is bitwise reproducible, and the diagonal matches sigma on
    sampled unit vectors."""
    torch = _torch()
    import paper_2609_09990_amd as pk
    h, B, e0 = synth.make_hamiltonian(20, 120, 0)
    sol = pk.Solver(pk.Problem(h, B, 10, 10, e0), M=1024, tol=1e-8)
    for k in range(9):
        sol.step(k, 0)
    k = 9
    e, tau, ok = sol.step(k, 0)
    assert ok
    n = sol.prepare(k)
    print(f"CAS(20,20) M=1024 k={k}: |psi| = {n}", flush=True)
    g = torch.Generator(device="cpu").manual_seed(7)
    x = torch.randn(n, dtype=torch.float64, generator=g).cuda()
    y = torch.randn(n, dtype=torch.float64, generator=g).cuda()
    hx, hy, hx2 = torch.zeros_like(x), torch.zeros_like(x), torch.zeros_like(x)
    sol.sigma(k, x, hx)
    sol.sigma(k, y, hy)
    sol.sigma(k, x, hx2)
    torch.cuda.synchronize()
    a, b = float(torch.dot(x, hy)), float(torch.dot(y, hx))
    assert abs(a - b) <= 1e-12 * float(torch.norm(hx)) * float(torch.norm(y)), (a, b)
    assert torch.equal(hx, hx2)
    d = torch.zeros_like(x)
    sol.diag(k, d)
    idx = torch.randint(0, n, (4,), generator=g).tolist()
    for i in idx:
        ei = torch.zeros_like(x)
        ei[i] = 1.0
        hi = torch.zeros_like(x)
        sol.sigma(k, ei, hi)
        torch.cuda.synchronize()
        assert abs(float(hi[i]) - float(d[i])) <= 1e-11 * max(1.0, abs(float(d[i])))
