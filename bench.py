"""Benchmark of the two-site DMRG sigma path on one MI355X.

Workload: CAS(20,20) active space (20 orbitals, 10 alpha + 10 beta electrons,
S_z = 0), 120 Cholesky vectors, bond dimension M = 1024, synthetic integrals
(seed 0).  Setup: a left-to-right half sweep from a random right-canonical MPS
up to the middle bond.  A step is one full two-site DMRG step at the middle bond
(sites 9, 10): Davidson on H_eff (fp64, tol 1e-8), SVD truncation, environment
update; steps alternate direction so every step re-solves the same bond.

Prints one JSON line (rank 0).  `value` = the sigma and environment-update
flops the kernels execute (unpadded block products) over the timed steps' wall
time.  The sweep time ("sweep") is the third full sweep (2(L-1) two-site steps
from site 0) of a fresh solver, timed end to end; step plans are rebuilt
whenever a step's outer bonds changed since its last visit.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sigma TFLOP/s + sweep s, CAS(20,20) M=1024; learned vs plain time to 1e-8 Ha"
N_ORB, N_CHOL, M, SEED = 20, 120, 1024, 0
MID = N_ORB // 2 - 1
PEAK_FP64 = 78.6  # TFLOP/s, MI355X dense FP64 matrix
# HBM bytes per launch of the dominant kernel from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE
# runs (profiles/sigma_step_kernels_cas20_m1024_fp64_counters.md), scaled by the same counters on a
# plain copy (fetch x2.0, write x1.0); set to None whenever that kernel changes.
TRAFFIC = 2.49e10


def _host_info():
    """Host CPU model, logical CPUs and the BLAS thread count the oracle runs with."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count()
    return model, os.cpu_count(), threads


def cpu_baseline(mps, h, B, gpu_sigma_ms, seconds=15.0):
    """The block-sparse oracle (its own MPO and environments, plain NumPy) timed
    on the host at the benched step: the GPU's MPS (dmrg_export_mps) at the
    middle bond of CAS(20,20), N_Q = 120, M = 1024.  Its environments are built
    first (untimed); then sigma output blocks of a seeded random two-site
    vector are computed one by one for about `seconds`.  value = the oracle's
    own matrix-product flops over its time; the full-sigma time is estimated
    from the sampled share of the output elements."""
    import numpy as np
    from oracle import blocks
    from oracle import mpo as om
    t0 = time.time()
    ts = blocks.TwoSite(om.build_mpo(h, B), mps, MID)
    setup_s = time.time() - t0
    print(f"# cpu baseline: oracle MPO and environments {setup_s:.0f} s", file=sys.stderr, flush=True)
    out = ts.output_blocks()
    size = {key: ts.bl.dim(key[0]) * ts.br.dim(key[2]) for key in out}
    total = sum(size.values())
    n = sum(size.values())
    psi = np.random.default_rng(23).standard_normal(n)
    order = np.random.default_rng(29).permutation(len(out))
    flops, done, elems = [0.0], 0, 0
    t1 = time.time()
    for i in order:
        key = out[i]
        ts.sigma(psi, blocks=[key], flops=flops)
        done += 1
        elems += size[key]
        if time.time() - t1 > seconds:
            break
    dt = time.time() - t1
    model, ncpu, threads = _host_info()
    return {"value": flops[0] / dt / 1e12, "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"block-sparse oracle sigma (own MPO, own environments from the GPU's exported MPS) at the "
                      f"benched step (CAS(20,20) N_Q=120 M=1024, sites {MID},{MID + 1}): {done} of {len(out)} "
                      f"output blocks ({elems} of {total} elements) in {dt:.1f} s; rate = the oracle's own "
                      f"matrix-product flop count of those blocks ({flops[0]:.3e}) over that time",
            "host": {"cpu_model": model, "logical_cpus": ncpu, "blas_threads": threads},
            "setup_s": setup_s,
            "sigma_seconds_est": dt * total / max(elems, 1),
            "gpu_sigma_ms": gpu_sigma_ms}


def precision_form(pk, sol, torch, direction, e_ref, fp64_ms, out):
    """Precision form at the bench bond: sigma in FP32 / BF16 on the matrix cores
    (fp32 accumulation), converged on an fp64 residual; energy against the FP64
    step's Ritz value, time against the FP64 step."""
    res = {}
    for name, prec in (("fp32", 1), ("bf16", 2)):
        sol.set_precision(prec)
        # one untimed step resolves this precision's plans (as the FP64 warm-up does)
        sol.step(MID, direction)
        direction ^= 1
        s0 = sol.stats()
        torch.cuda.synchronize()
        t0 = time.time()
        err, ok_all = 0.0, True
        for _ in range(2):
            e, tau, ok = sol.step(MID, direction)
            direction ^= 1
            err = max(err, abs(float(e[0]) - e_ref))
            ok_all = ok_all and ok
        torch.cuda.synchronize()
        ms = (time.time() - t0) / 2 * 1e3
        s1 = sol.stats()
        res[name] = {"ms_per_step": ms, "speedup_vs_fp64": fp64_ms / ms, "energy_err_vs_fp64": err,
                     "converged": ok_all, "matvecs_per_step": (s1["matvecs"] - s0["matvecs"]) / 2,
                     "lowp_matvecs_per_step": (s1["lowp_matvecs"] - s0["lowp_matvecs"]) / 2,
                     "fp64_refinements": s1["refinements"] - s0["refinements"],
                     "sigma_ms_per_step": (s1["sigma_a_ms"] + s1["sigma_b_ms"] - s0["sigma_a_ms"] - s0["sigma_b_ms"]) / 2}
        print(f"# precision {name}: {ms:.0f} ms/step dE={err:.2e}", file=sys.stderr, flush=True)
    sol.set_precision(0)
    res["three_roots"] = precision_three_roots(pk, torch)
    out["precision_form"] = res
    return direction


def precision_three_roots(pk, torch):
    """Per-state error of the precision form: 3 state-averaged roots at the bench
    bond (CAS(20,20), N_Q = 120, M = 1024), one FP64 half sweep to the middle,
    then the middle step from that same MPS in FP64 and in FP32."""
    import synth
    h, B, e0 = synth.make_hamiltonian(N_ORB, N_CHOL, SEED)
    sol = pk.Solver(pk.Problem(h, B, N_ORB // 2, N_ORB // 2, e0), M=M, n_states=3, tol=1e-8)
    for k in range(MID):
        sol.step(k, 0)
    start = sol.export_mps()
    res = {}
    for name, prec in (("fp64", 0), ("fp32", 1)):
        sol.set_mps(start["bonds"], start["sites"])
        sol.set_precision(prec)
        sol.prepare(MID)
        s0 = sol.stats()
        torch.cuda.synchronize()
        t0 = time.time()
        e, tau, ok = sol.step(MID, 0)
        torch.cuda.synchronize()
        s1 = sol.stats()
        res[name] = {"ms": (time.time() - t0) * 1e3, "energies": [float(x) for x in e], "converged": bool(ok),
                     "matvecs": s1["matvecs"] - s0["matvecs"], "lowp_matvecs": s1["lowp_matvecs"] - s0["lowp_matvecs"]}
    res["fp32"]["energy_err_per_state"] = [abs(a - b) for a, b in zip(res["fp32"]["energies"], res["fp64"]["energies"])]
    res["fp32"]["speedup_vs_fp64"] = res["fp64"]["ms"] / res["fp32"]["ms"]
    print(f"# precision, 3 roots: fp32 |dE| {res['fp32']['energy_err_per_state']}, "
          f"{res['fp32']['speedup_vs_fp64']:.2f}x", file=sys.stderr, flush=True)
    del sol
    return res


def train_preconditioner(pk, torch):
    """Learned preconditioner trained on the GPU (the library's forward, backward
    and Adam kernels) on triples the solver records from diagonal-preconditioned
    sweeps: 20 Hamiltonians of the same generator (seeds 1-20, held out from the
    benched seed 0), CAS(12,12) / CAS(14,14) at M = 256 and CAS(16,16) at M = 512
    in turn, 1024 amplitudes per triple."""
    import synth
    from paper_2609_09990_amd import precond as pc
    t0 = time.time()
    Xs, Ts = [], []
    for seed in range(1, 21):
        n = (12, 14, 16)[seed % 3]
        hh, BB, ee = synth.make_hamiltonian(n, 6 * n, seed)
        X, T = pc.collect_triples([(hh, BB, ee)], n // 2, n // 2, M=512 if n == 16 else 256, sweeps=1, sample=1024,
                                  capacity=5000, tol=1e-8)
        Xs.append(X)
        Ts.append(T)
        print(f"# learned: triples from seed {seed} (CAS({n},{n})) done", file=sys.stderr, flush=True)
    X, T = torch.cat(Xs), torch.cat(Ts)
    collect_s = time.time() - t0
    net = pk.MLP(8, 256, seed=0)
    hist = pc.train(net, X, T, steps=800, batch=64, lr=1e-3)
    torch.cuda.synchronize()
    train_s = time.time() - t0
    info = {"seconds": train_s, "collect_seconds": collect_s, "hamiltonians": 20, "triples": int(X.shape[0]),
            "sample": int(X.shape[1]), "loss_first": float(hist[:20].mean()), "loss_last": float(hist[-20:].mean()),
            "diag_candidate_loss": pc.diag_baseline_loss(X, T)}
    print(f"# learned: trained on {X.shape[0]} triples in {train_s:.0f} s, loss {hist[-20:].mean():.3f} "
          f"(diagonal candidate {info['diag_candidate_loss']:.3f})", file=sys.stderr, flush=True)
    del X, T, Xs, Ts
    return net, info


def learned_form(pk, sol, torch, direction, e_ref, net, info, out):
    """The bench bond's step (Davidson to a residual of 1e-8: energy within 1e-8
    Ha of the FP64 reference) with each preconditioner and sigma precision."""
    res = {"training": info}
    for name, prec, mode in (("fp64_diag", 0, 0), ("fp64_learned", 0, 1), ("fp32_diag", 1, 0),
                             ("fp32_learned", 1, 1)):
        sol.set_precision(prec)
        sol.set_precond(mode, net if mode else None)
        s0 = sol.stats()
        torch.cuda.synchronize()
        t1 = time.time()
        e, tau, ok = sol.step(MID, direction)
        direction ^= 1
        torch.cuda.synchronize()
        s1 = sol.stats()
        res[name] = {"ms": (time.time() - t1) * 1e3, "matvecs": s1["matvecs"] - s0["matvecs"],
                     "lowp_matvecs": s1["lowp_matvecs"] - s0["lowp_matvecs"],
                     "energy_err_vs_fp64": abs(float(e[0]) - e_ref), "converged": bool(ok),
                     "fallbacks": s1["fallbacks"] - s0["fallbacks"]}
        print(f"# {name}: {res[name]['ms']:.0f} ms, {res[name]['matvecs']:.0f} matvecs", file=sys.stderr, flush=True)
    sol.set_precision(0)
    sol.set_precond(0, None)
    res["time_to_1e-8"] = time_to_target(pk, torch, net)
    out["learned_form"] = res
    return direction


def config5(pk, torch, net):
    """CAS(24,24), N_Q = 160, M = 2048 (the learned-preconditioner configuration):
    an FP64 left-to-right half sweep from the seeded start reaches the middle
    bond; its MPS is the common start of every method.  The reference energy is
    the middle-bond solve in FP64 with Davidson tol 1e-10.  Each method then
    solves the same bond from the same MPS and guess with tol 1e-8 (energy
    error ~ r^2 / gap, far below 1e-8 Ha); wall time of the step (Davidson,
    truncation and environment update; environments prepared beforehand) and
    matvecs."""
    import synth
    n, nq, Mb = 24, 160, 2048
    mid = n // 2 - 1
    h, B, e0 = synth.make_hamiltonian(n, nq, SEED)
    prob = pk.Problem(h, B, n // 2, n // 2, e0)
    sol = pk.Solver(prob, M=Mb, tol=1e-8)
    t0 = time.time()
    for k in range(mid):
        sol.step(k, 0)
        print(f"# config 5 half sweep step {k} done", file=sys.stderr, flush=True)
    half_s = time.time() - t0
    start = sol.export_mps()
    res = {"workload": "CAS(24,24) N_Q=160 M=2048 seed 0, middle bond after an FP64 half sweep",
           "half_sweep_s": half_s, "psi": int(sol.prepare(mid))}
    ref = pk.Solver(prob, M=Mb, tol=1e-10)
    ref.set_mps(start["bonds"], start["sites"])
    ref.prepare(mid)
    e, _, ok = ref.step(mid, 0)
    e_ref = float(e[0])
    res["e_ref"] = e_ref
    res["ref_converged"] = bool(ok)
    del ref
    print(f"# config 5 reference E = {e_ref:.10f}", file=sys.stderr, flush=True)
    for name, prec, mode in (("fp64_diag", 0, 0), ("fp32_diag", 1, 0), ("fp32_learned", 1, 1),
                             ("fp64_learned", 0, 1)):
        sol.set_mps(start["bonds"], start["sites"])
        sol.set_precision(prec)
        sol.set_precond(mode, net if mode else None)
        sol.prepare(mid)
        s0 = sol.stats()
        torch.cuda.synchronize()
        t1 = time.time()
        e, tau, ok = sol.step(mid, 0)
        torch.cuda.synchronize()
        s1 = sol.stats()
        res[name] = {"seconds": time.time() - t1, "matvecs": s1["matvecs"] - s0["matvecs"],
                     "lowp_matvecs": s1["lowp_matvecs"] - s0["lowp_matvecs"],
                     "energy_err": abs(float(e[0]) - e_ref), "reached_1e-8": abs(float(e[0]) - e_ref) <= 1e-8,
                     "converged": bool(ok), "fallbacks": s1["fallbacks"] - s0["fallbacks"]}
        print(f"# config 5 {name}: {res[name]['seconds']:.2f} s, {res[name]['matvecs']:.0f} matvecs, "
              f"dE {res[name]['energy_err']:.1e}", file=sys.stderr, flush=True)
    base = res["fp64_diag"]["seconds"]
    for name in ("fp32_diag", "fp32_learned", "fp64_learned"):
        res[name]["speedup_vs_fp64_diag"] = base / res[name]["seconds"]
    del sol
    return res


def time_to_target(pk, torch, net):
    """Time to 1e-8 Ha: CAS(16,16), N_Q = 96, M = 512 (seed 0, held out from the
    training seeds).  The reference energy is an FP64 run with Davidson tol 1e-10
    swept until two sweeps agree to 1e-11 Ha.  Each method then starts from the
    same seeded initial MPS (Davidson tol 1e-8) and its clock stops at the first
    sweep boundary whose energy is within 1e-8 Ha of the reference."""
    import synth
    hh, BB, ee = synth.make_hamiltonian(16, 96, 0)
    prob = pk.Problem(hh, BB, 8, 8, ee)
    ref = pk.Solver(prob, M=512, tol=1e-10)
    e_prev, e_ref = None, None
    for _ in range(14):
        e, tau, ok = ref.sweep(1)
        e_ref = float(e[0])
        print(f"# to 1e-8 Ha: reference sweep E = {e_ref:.12f}", file=sys.stderr, flush=True)
        if e_prev is not None and abs(e_ref - e_prev) < 1e-11:
            break
        e_prev = e_ref
    del ref
    res = {"workload": "CAS(16,16) N_Q=96 M=512 seed 0", "e_ref": e_ref}
    for name, prec, mode in (("fp64_diag", 0, 0), ("fp32_diag", 1, 0), ("fp32_learned", 1, 1),
                             ("fp64_learned", 0, 1)):
        sol = pk.Solver(prob, M=512, tol=1e-8, precision=prec)
        sol.set_precond(mode, net if mode else None)
        wall, sweeps, err = 0.0, 0, None
        s0 = sol.stats()
        for _ in range(10):
            torch.cuda.synchronize()
            t0 = time.time()
            e, tau, ok = sol.sweep(1)
            torch.cuda.synchronize()
            wall += time.time() - t0
            sweeps += 1
            err = abs(float(e[0]) - e_ref)
            if err <= 1e-8:
                break
        s1 = sol.stats()
        res[name] = {"seconds": wall, "sweeps": sweeps, "matvecs": s1["matvecs"] - s0["matvecs"],
                     "reached": bool(err is not None and err <= 1e-8), "final_err": err}
        print(f"# to 1e-8 Ha, {name}: {wall:.1f} s, {sweeps} sweeps, {res[name]['matvecs']:.0f} matvecs",
              file=sys.stderr, flush=True)
        del sol
    base = res["fp64_diag"]["seconds"]
    for name in ("fp32_diag", "fp32_learned", "fp64_learned"):
        res[name]["speedup_vs_fp64_diag"] = base / res[name]["seconds"] if res[name]["seconds"] > 0 else None
    return res


def adjoint_form(sol, torch, h, B, e_core, out):
    """Adjoint form: dE/dh and dE/dB^Q of the current MPS (dmrg_grad) at the bench
    size, with the properties that hold for any state as checks."""
    import numpy as np
    s0 = sol.stats()
    torch.cuda.synchronize()
    t0 = time.time()
    dh, dB, e = sol.grad()
    dt = time.time() - t0
    s1 = sol.stats()
    euler = float(np.sum(h * dh) + 0.5 * np.sum(B * dB))
    out["adjoint_form"] = {"seconds": dt, "tflops": (s1["grad_flops"] - s0["grad_flops"]) / dt / 1e12,
                           "energy": float(e[0]), "trace_dE_dh": float(np.trace(dh)),
                           "euler_residual": abs(euler - (float(e[0]) - e_core)),
                           "dE_dh_asymmetry": float(np.abs(dh - dh.T).max())}
    print(f"# adjoint: {dt:.1f} s", file=sys.stderr, flush=True)


def oracle_beside(pk, torch):
    """The CPU oracle timed beside the device on the same inputs (small cases the
    oracle finishes in seconds): 1-/2-RDMs at CAS(8,8), the three-body density at
    CAS(5,5), mutual information at CAS(6,6); random CI vectors."""
    import numpy as np
    import synth
    from oracle import fci, orbital
    out = {}
    for name, (n, na, nb) in (("rdm12_cas8", (8, 4, 4)), ("rdm3_cas5", (5, 3, 2)), ("mutual_information_cas6", (6, 3, 3))):
        h, B, e0 = synth.make_hamiltonian(n, 8, 0)
        prob = pk.Problem(h, B, na, nb, e0)
        space = fci.DetSpace(n, na, nb)
        c = np.random.default_rng(n).normal(size=space.shape)
        dc = torch.from_numpy(c).cuda()
        t0 = time.time()
        if name.startswith("rdm12"):
            g, G, _ = prob.ci_rdm12(dc)
        elif name.startswith("rdm3"):
            G = prob.ci_rdm3(dc)
        else:
            s1, G = prob.mutual_information(dc)
        t_gpu = time.time() - t0
        t0 = time.time()
        if name.startswith("rdm12"):
            rg, rG = fci.rdm12(space, c)
        elif name.startswith("rdm3"):
            rG = fci.rdm3(space, c, c)
        else:
            rs1, rG = orbital.mutual_information(space, c)
        t_cpu = time.time() - t0
        out[name] = {"gpu_s": t_gpu, "oracle_cpu_s": t_cpu, "max_abs_diff": float(np.abs(G - rG).max())}
        print(f"# oracle beside {name}: gpu {t_gpu:.3f} s, oracle {t_cpu:.2f} s", file=sys.stderr, flush=True)
    return out


def next_rows(pk, torch):
    """The rows beyond the step, timed on their own workloads (synthetic
    integrals, the sizes of the paper's validation active spaces):
    * excited states: the three lowest CAS(12,12) roots (N_Q = 64, M = 512) by
      penalty deflation with the diagonal and with the shift-and-invert
      preconditioner: wall time, sweeps, energy difference; the same for the
      near-degenerate lowest CAS(8,8) roots (N_Q = 32, M = 256);
    * determinant space at CAS(12,12): MPS to CI vector, 1-/2-RDMs (the
      (n^2+1)^2 x N_det product on the fp64 MFMA kernel: rate), V c and the
      fused four-body contraction as the three-body density of (c, V c), orbital
      mutual information and the Fiedler order;
    * stationarity at truncated M: one-site sweeps of CAS(8,8) (N_Q = 32) at
      M = 24, where the two-site fixed point discards ~1e-2."""
    import numpy as np
    import synth
    res = {}
    h, B, e0 = synth.make_hamiltonian(12, 64, 0)
    prob = pk.Problem(h, B, 6, 6, e0)
    ex = {}
    for mode in (0, 3):
        torch.cuda.synchronize()
        t0 = time.time()
        r = pk.excited_states(prob, 3, M=512, tol=1e-9, sweeps=3, conv_tol=1e-9, precond=mode)
        dt = time.time() - t0
        ex[mode] = (dt, r["energies"], sum(run["sweeps"] for run in r["runs"]))
        print(f"# excited states precond {mode}: {dt:.1f} s", file=sys.stderr, flush=True)
    res["excited_cas12_m512"] = {
        "roots": 3, "seconds_diag": ex[0][0], "seconds_shift_invert": ex[3][0],
        "speedup_shift_invert": ex[0][0] / ex[3][0], "energies": [float(x) for x in ex[3][1]],
        "max_abs_energy_difference": float(np.max(np.abs(ex[0][1] - ex[3][1]))),
        "sweeps_diag": ex[0][2], "sweeps_shift_invert": ex[3][2]}
    # near-degenerate roots (the two lowest CAS(8,8) roots are 5 mHa apart)
    h8, B8, e8 = synth.make_hamiltonian(8, 32, 0)
    p8 = pk.Problem(h8, B8, 4, 4, e8)
    nd = {}
    for mode in (0, 3):
        torch.cuda.synchronize()
        t0 = time.time()
        r = pk.excited_states(p8, 3, M=256, tol=1e-10, sweeps=3, conv_tol=1e-11, precond=mode)
        nd[mode] = (time.time() - t0, r["energies"])
    res["excited_cas8_near_degenerate"] = {
        "roots": 3, "gap_lowest_ha": float(nd[0][1][1] - nd[0][1][0]), "seconds_diag": nd[0][0],
        "seconds_shift_invert": nd[3][0], "speedup_shift_invert": nd[0][0] / nd[3][0],
        "max_abs_energy_difference": float(np.max(np.abs(nd[0][1] - nd[3][1])))}
    print(f"# near-degenerate roots: diag {nd[0][0]:.2f} s, shift-invert {nd[3][0]:.2f} s", file=sys.stderr,
          flush=True)
    sol = pk.Solver(prob, M=1024, tol=1e-9)
    sol.sweep(3)
    na, nb = prob.ci_dims()
    torch.cuda.synchronize()
    t0 = time.time()
    c = sol.mps_to_ci()
    torch.cuda.synchronize()
    t_ci = time.time() - t0
    t0 = time.time()
    g, G, ov = prob.ci_rdm12(c)
    t_12 = time.time() - t0
    rows = 12 * 12 + 1
    f12 = 2.0 * rows * rows * na * nb
    t0 = time.time()
    vc = prob.ci_apply_v(c)
    torch.cuda.synchronize()
    t_v = time.time() - t0
    t0 = time.time()
    F = prob.ci_rdm3(c, vc)
    t_3 = time.time() - t0
    f3 = 2.0 * rows * (144 * rows) * na * nb
    t0 = time.time()
    s1, I = prob.mutual_information(c)
    order, _ = pk.fiedler_order(I)
    t_mi = time.time() - t0
    e_rdm = float(np.sum(h * g) + 0.5 * np.einsum("Qpq,Qrs,pqrs->", B, B, G)) / ov + e0
    res["determinant_space_cas12"] = {
        "n_det": na * nb, "mps_to_ci_s": t_ci, "rdm12_s": t_12, "rdm12_gemm_flops": f12,
        "rdm12_tflops": f12 / t_12 / 1e12, "apply_v_s": t_v, "rdm3_of_c_vc_s": t_3, "rdm3_gemm_flops": f3,
        "rdm3_tflops": f3 / t_3 / 1e12, "mutual_information_and_order_s": t_mi,
        "energy_from_rdm_minus_dmrg": e_rdm - float(sol.energy()[0]),
        "fused_trace_check": float(np.einsum("pprrtt->", F) / (12 ** 3 * float((c * vc).sum())) - 1.0)}
    res["determinant_space_cas12"]["rdm12_frac_fp64_peak"] = f12 / t_12 / 1e12 / PEAK_FP64
    res["determinant_space_cas12"]["rdm3_frac_fp64_peak"] = f3 / t_3 / 1e12 / PEAK_FP64
    print(f"# determinant space: rdm12 {t_12:.2f} s, rdm3(c, Vc) {t_3:.2f} s", file=sys.stderr, flush=True)
    res["oracle_beside"] = oracle_beside(pk, torch)
    del sol
    # mutual information and order from the MPS itself at the bench active space (M = 256)
    h20, B20, e20 = synth.make_hamiltonian(N_ORB, N_CHOL, SEED)
    s20 = pk.Solver(pk.Problem(h20, B20, N_ORB // 2, N_ORB // 2, e20), M=256, tol=1e-7)
    s20.sweep(2)
    torch.cuda.synchronize()
    t0 = time.time()
    rho, s1, I = s20.orbital_entanglement()
    order, _ = pk.fiedler_order(I)
    t_mi = time.time() - t0
    res["ordering_cas20_m256"] = {"orbital_entanglement_s": t_mi, "order": [int(x) for x in order],
                                  "s1_max": float(s1.max()), "I_max": float(I.max()),
                                  "trace_error": float(np.abs(np.trace(rho, axis1=1, axis2=2) - 1).max())}
    print(f"# ordering at CAS(20,20) M=256: {t_mi:.2f} s", file=sys.stderr, flush=True)
    del s20
    h8, B8, e8 = synth.make_hamiltonian(8, 32, 0)
    st = pk.Solver(pk.Problem(h8, B8, 4, 4, e8), M=24, tol=1e-11)
    e2 = st.sweep(6)[0][0]
    torch.cuda.synchronize()
    t0 = time.time()
    out = []
    for _ in range(20):
        e, r, ok = st.stationarize(1)
        out.append(r)
    dt = time.time() - t0
    res["stationarize_cas8_m24"] = {"seconds_per_sweep": dt / 20, "energy_two_site": float(e2),
                                    "energy_after_20": float(e), "tangent_residual_every_5": out[::5] + [out[-1]]}
    print(f"# stationarize: {dt / 20:.2f} s per sweep", file=sys.stderr, flush=True)
    return res


def diff_form(pk, torch):
    """Differentiation form: CAS(16,16), N_Q = 96, M = 512, 2 state-averaged roots
    (seed 0), 4 sweeps.  Per-state gradients of the final MPS (time), and the
    central finite difference (step 1e-5) of each root's energy along a random
    symmetric direction of (h, B), each side a full DMRG run from the same
    start: at truncated bond the two differ by an amount that tracks the
    discarded weight (the MPS is not stationary in the full tangent space)."""
    import numpy as np
    import synth
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

    t0 = time.time()
    sol, e, tau, ok = run(h, B)
    run_s = time.time() - t0
    res = {"config": "CAS(16,16) N_Q=96 M=512 2 states, 4 sweeps", "dmrg_s": run_s, "energies": e.tolist(),
           "tau_last_sweep": tau, "converged": bool(ok), "states": []}
    ep = run(h + eps * Dh, B + eps * DB)[1]
    em = run(h - eps * Dh, B - eps * DB)[1]
    for r in range(2):
        w = np.zeros(2)
        w[r] = 1.0
        torch.cuda.synchronize()
        t1 = time.time()
        dh, dB, _ = sol.grad(w)
        gs = time.time() - t1
        analytic = float(np.sum(dh * Dh) + np.sum(dB * DB))
        fd = float((ep[r] - em[r]) / (2 * eps))
        res["states"].append({"grad_s": gs, "analytic": analytic, "finite_difference": fd,
                              "gap": abs(analytic - fd), "trace_dE_dh": float(np.trace(dh))})
    print(f"# diff form: {res}", file=sys.stderr, flush=True)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sweep", action="store_true", help="skip the timed full sweep")
    ap.add_argument("--no-forms", action="store_true", help="skip the precision, learned and adjoint forms")
    ap.add_argument("--no-config5", action="store_true", help="skip the CAS(24,24) M=2048 comparison")
    ap.add_argument("--no-next", action="store_true",
                    help="skip the excited-state, determinant-space and stationarity timings")
    ap.add_argument("--rows-only", action="store_true",
                    help="run only those timings and print them as one JSON line (for profiling)")
    ap.add_argument("--diff-form", action="store_true",
                    help="also run the differentiation-form configuration (CAS(16,16), M=512, 2 states)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path (sigma would shard over middle-cut "
              "channels with one all-reduce per matvec)", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2609_09990_amd as pk
    import synth

    if args.rows_only:
        print(json.dumps({"next_rows": next_rows(pk, torch)}), flush=True)
        return
    h, B, e0 = synth.make_hamiltonian(N_ORB, N_CHOL, SEED)
    prob = pk.Problem(h, B, N_ORB // 2, N_ORB // 2, e0)
    sol = pk.Solver(prob, M=M, tol=1e-8, precision=args.precision)
    t_setup = time.time()
    for k in range(MID):
        sol.step(k, 0)
        print(f"# setup step {k} done", file=sys.stderr, flush=True)
    # one step at the bench bond in each direction: the step plan and both
    # environment-update plans exist before the warm-up and timed steps
    sol.step(MID, 0)
    sol.step(MID, 1)
    t_setup = time.time() - t_setup
    direction = 0
    for w in range(args.warmup):
        sol.step(MID, direction)
        direction ^= 1
        print(f"# warmup step {w} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    sol.set_kernel_tag(1)  # timed sigma launches use their own kernel names (profile separation)
    s0 = sol.stats()
    t0 = time.time()
    energies = []
    for i in range(args.steps):
        e, tau, ok = sol.step(MID, direction)
        direction ^= 1
        energies.append(float(e[0]))
        print(f"# timed step {i} E={e[0]:.10f} tau={tau:.2e} converged={ok}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.time() - t0
    s1 = sol.stats()
    sol.set_kernel_tag(0)  # only the timed steps above use the tagged kernel names
    d = {k: s1[k] - s0[k] for k in s1}
    # flops the kernels execute (unpadded block products of the merged / trimmed
    # plan); the factorisation's algorithmic count is reported beside them
    sig_flops = d["sigma_a_flops_exec"] + d["sigma_b_flops_exec"]
    sig_flops_alg = d["sigma_a_flops"] + d["sigma_b_flops"]
    tot_flops = sig_flops + d["env_flops"]
    ms_per_step = 1e3 * wall / args.steps
    nmv = max(d["matvecs"], 1)
    # dominant kernel: the long-K block GEMM of sigma (phase B); HIP-event time per launch of
    # the GEMM kernel alone (events on the solver stream around that launch)
    b_launch_ms = d["sigma_b_gemm_ms"] / nmv
    b_flops = d["sigma_b_flops_exec"] / nmv
    b_achieved = b_flops / (b_launch_ms * 1e-3) / 1e12 if b_launch_ms > 0 else 0.0
    mps_bench = sol.export_mps()  # the benched state, for the CPU oracle baseline
    out = {
        "metric": METRIC,
        "value": tot_flops / wall / 1e12,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ["f64", "f32", "bf16"][args.precision],
        "data": "synthetic",
        "config": {"workload": "CAS(20,20) two-site DMRG step at the middle bond", "n_orb": N_ORB,
                   "n_chol": N_CHOL, "M": M, "davidson_tol": 1e-8, "seed": SEED},
        "sigma_kernel_tflops": sig_flops / ((d["sigma_a_ms"] + d["sigma_b_ms"]) * 1e-3) / 1e12,
        # the same sigma time over the factorisation's algorithmic count (every T_X
        # column block, every unmerged item)
        "sigma_kernel_tflops_algorithmic": sig_flops_alg / ((d["sigma_a_ms"] + d["sigma_b_ms"]) * 1e-3) / 1e12,
        "sigma_ms_per_matvec": (d["sigma_a_ms"] + d["sigma_b_ms"]) / nmv,
        "sigma_flops_per_matvec": sig_flops / nmv,
        "matvecs_per_step": nmv / args.steps,

        "breakdown_ms_per_step": {"sigma": (d["sigma_a_ms"] + d["sigma_b_ms"]) / args.steps,
                                  "env": d["env_ms"] / args.steps, "svd": d["svd_ms"] / args.steps,
                                  "prepare_wall": d["prepare_ms"] / args.steps,
                                  "plan_resolve_wall": d["resolve_ms"] / args.steps,
                                  "davidson_wall": d["davidson_ms"] / args.steps},
        "setup_s": t_setup,
        "energy_last": energies[-1] if energies else None,
        "plan_reuse_per_step": (d["plan_hits"]) / args.steps,
        "roofline": {"bound": "mfma", "kernel": "gemm_wg<double, 4> (sigma phase B, timed launches)",
                     "achieved": b_achieved, "peak": PEAK_FP64, "unit": "TFLOP/s",
                     "frac": b_achieved / PEAK_FP64, "traffic": TRAFFIC,
                     "launch_ms": b_launch_ms, "flops_per_launch": b_flops,
                     "algorithmic_flops_per_launch": d["sigma_b_flops"] / nmv},
    }
    # measured device ceilings (register-only fp64 MFMA loop, 2 GiB streaming copy)
    mf, cp = pk.measure_peaks(1 << 31)
    out["measured_peaks"] = {"fp64_mfma_tflops": mf, "copy_gbs": cp,
                             "phase_b_frac_of_measured_mfma": b_achieved / mf if mf > 0 else None}
    print(f"# measured fp64 MFMA {mf:.1f} TFLOP/s, copy {cp:.0f} GB/s", file=sys.stderr, flush=True)
    net = None
    if not args.no_forms:
        direction = precision_form(pk, sol, torch, direction, energies[-1], ms_per_step, out)
        net, info = train_preconditioner(pk, torch)
        direction = learned_form(pk, sol, torch, direction, energies[-1], net, info, out)
    if not args.no_sweep:
        # sweep time: the third full sweep (2(L-1) two-site steps from site 0) of a
        # fresh solver at steady M = 1024, timed end to end
        swp = pk.Solver(prob, M=M, tol=1e-8)
        for i in range(2):
            swp.sweep(1)
            print(f"# sweep {i + 1} done (untimed)", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        s2 = swp.stats()
        t0 = time.time()
        e, tau, ok = swp.sweep(1)
        torch.cuda.synchronize()
        sweep_s = time.time() - t0
        s3 = swp.stats()
        dd = {k: s3[k] - s2[k] for k in s3}
        out["sweep"] = {"seconds": sweep_s, "which": "third sweep of a fresh solver", "steps": 2 * (N_ORB - 1),
                        "energy": float(e[0]), "tau_max": tau, "converged": bool(ok), "matvecs": dd["matvecs"],
                        "plan_reuse": dd["plan_hits"],
                        "breakdown_s": {"sigma": (dd["sigma_a_ms"] + dd["sigma_b_ms"]) / 1e3,
                                        "env": dd["env_ms"] / 1e3, "svd": dd["svd_ms"] / 1e3,
                                        "davidson_other": (dd["davidson_ms"] - dd["sigma_a_ms"]
                                                           - dd["sigma_b_ms"]) / 1e3,
                                        "prepare_wall": dd["prepare_ms"] / 1e3},
                        "tflops": (dd["sigma_a_flops_exec"] + dd["sigma_b_flops_exec"] + dd["env_flops"])
                        / sweep_s / 1e12}
        print(f"# sweep 3: {sweep_s:.1f} s E={e[0]:.10f}", file=sys.stderr, flush=True)
        if not args.no_forms:
            adjoint_form(swp, torch, h, B, e0, out)
        del swp
    if args.diff_form:
        out["diff_form"] = diff_form(pk, torch)
    if not args.no_next:
        out["next_rows"] = next_rows(pk, torch)
    if net is not None and not args.no_config5:
        del sol
        out["config5"] = config5(pk, torch, net)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(mps_bench, h, B, out["sigma_ms_per_matvec"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
