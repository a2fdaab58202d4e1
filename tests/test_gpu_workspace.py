"""Solver device memory in a torch-allocated workspace (dmrg_workspace_query /
dmrg_workspace_attach): the same results as with the library's own buffers, no
hipMalloc on the solver path once attached, growth after DMRG_ENOMEM, and a
re-attach in the middle of a run."""
import json
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fci_energies.json")


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_sweep_in_torch_workspace_matches_and_allocates_nothing():
    torch = _torch()
    import paper_2609_09990_amd as pk
    h, B, e0 = synth.make_hamiltonian(8, 32, 0)
    prob = pk.Problem(h, B, 4, 4, e0)
    ref = pk.Solver(prob, M=256, tol=1e-10)
    e_ref, _, ok_ref = ref.sweep(2)
    sol = pk.Solver(prob, M=256, tol=1e-10, workspace=True)
    size = sol._ws.numel()
    e, tau, ok = sol.sweep(2)
    st = sol.stats()
    print(f"workspace {size / 2**20:.0f} MiB, peak {st['workspace_peak_bytes'] / 2**20:.0f} MiB, "
          f"allocations since attach {st['device_allocs_since_attach']:.0f}", flush=True)
    assert ok and ok_ref
    assert np.array_equal(e, e_ref)  # the same kernels in the same order: bitwise equal
    assert st["device_allocs_since_attach"] == 0
    assert 0 < st["workspace_peak_bytes"] <= size
    fci = json.load(open(GOLD))["cas8_nq32_s0"]["energies"][0]
    assert abs(e[0] - fci) <= 1e-10


def test_workspace_grows_after_enomem_and_reattach_mid_run():
    torch = _torch()
    import paper_2609_09990_amd as pk
    h, B, e0 = synth.make_hamiltonian(8, 32, 0)
    prob = pk.Problem(h, B, 4, 4, e0)
    ref = pk.Solver(prob, M=64, tol=1e-10)
    e_ref = [ref.step(k, 0)[0][0] for k in range(7)]
    sol = pk.Solver(prob, M=64, tol=1e-10, workspace=2 << 20)  # 2 MiB: too small for a step
    # the step reports DMRG_ENOMEM, the binding queries, attaches a larger
    # workspace and runs the step again
    got = [sol.step(0, 0)[0][0]]
    assert sol._ws.numel() > (2 << 20)
    for k in range(1, 4):
        got.append(sol.step(k, 0)[0][0])
    # move the solver into a new, larger workspace in the middle of the sweep
    sol.attach_workspace(sol.workspace_query() * 2)
    for k in range(4, 7):
        got.append(sol.step(k, 0)[0][0])
    st = sol.stats()
    print("steps", np.array(got) - np.array(e_ref), "allocations since attach", st["device_allocs_since_attach"],
          flush=True)
    assert st["device_allocs_since_attach"] == 0
    assert np.max(np.abs(np.array(got) - np.array(e_ref))) <= 1e-9


def test_workspace_query_covers_a_half_sweep_cas12():
    """The estimate before any work covers a CAS(12,12), M = 512 half sweep, and
    after it the query asks for at least 1.25 times the peak."""
    torch = _torch()
    import paper_2609_09990_amd as pk
    h, B, e0 = synth.make_hamiltonian(12, 64, 0)
    sol = pk.Solver(pk.Problem(h, B, 6, 6, e0), M=512, tol=1e-9)
    q = sol.workspace_query()
    sol.attach_workspace(q)
    for k in range(6):
        sol.step(k, 0)
    st = sol.stats()
    print(f"estimate {q / 2**20:.0f} MiB, peak {st['workspace_peak_bytes'] / 2**20:.0f} MiB", flush=True)
    assert sol._ws.numel() == q  # no growth was needed
    assert st["workspace_peak_bytes"] <= q
    assert sol.workspace_query() >= 1.25 * st["workspace_peak_bytes"]
