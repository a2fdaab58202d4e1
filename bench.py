"""Benchmark of the two-site DMRG sigma path on one MI355X.

Workload: CAS(20,20) active space (20 orbitals, 10 alpha + 10 beta electrons,
S_z = 0), 120 Cholesky vectors, bond dimension M = 1024, synthetic integrals
(seed 0).  Setup: a left-to-right half sweep from a random right-canonical MPS
up to the middle bond.  A step is one full two-site DMRG step at the middle bond
(sites 9, 10): Davidson on H_eff (fp64, tol 1e-8), SVD truncation, environment
update; steps alternate direction so every step re-solves the same bond.

Prints one JSON line (rank 0).  `value` = algorithmic sigma + environment-update
TFLOP/s over the timed steps' wall time.  After the steps, one full sweep
(2(L-1) two-site steps from site 0) is timed end to end ("sweep"); step plans
are rebuilt whenever a step's outer bonds changed since its last visit.
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
# runs (profiles/sigma_phaseB_w32_cas20_m1024_fp64.md), scaled by the same counters on a
# plain copy (fetch x2.0, write x1.0); set to None whenever that kernel changes.
TRAFFIC = 4.291e10


def cpu_baseline(pk, torch):
    """The oracle's projected two-site sigma (determinant FCI through the MPS
    embedding) timed on the host for a bounded sample: CAS(8,8), 32 Cholesky
    vectors, M = 256, middle step, repeated for about 10 s; rate = the GPU
    planner's algorithmic flops of that same sigma / oracle seconds."""
    import numpy as np
    import synth
    from oracle import embed
    n, na, nq, Mb, k = 8, 4, 32, 256, 3
    h, B, e0 = synth.make_hamiltonian(n, nq, SEED)
    mps = synth.random_mps(n, na, na, Mb, seed=5)
    prob = pk.Problem(h, B, na, na, e0)
    sol = pk.Solver(prob, M=Mb)
    sol.set_mps(mps["bonds"], mps["sites"])
    sol.prepare(k)
    psi = synth.random_twosite(mps["bonds"], k, seed=11)
    d = torch.from_numpy(psi).cuda()
    o = torch.zeros_like(d)
    flops = sol.sigma(k, d, o)
    reps, t0 = 0, time.time()
    while True:
        embed.sigma_twosite(h, B, mps, k, psi, na, na, e0)
        reps += 1
        if time.time() - t0 > 10.0 or reps >= 200:
            break
    dt = (time.time() - t0) / reps
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count()
    return {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"oracle projected sigma (FCI via MPS embedding), CAS(8,8) N_Q=32 M=256 middle step, "
                      f"{reps} calls, {dt:.2f} s each; flops = GPU-plan algorithmic count {flops:.3e}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sweep", action="store_true", help="skip the timed full sweep")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (see DESIGN.md, sharding)",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2609_09990_amd as pk
    import synth

    h, B, e0 = synth.make_hamiltonian(N_ORB, N_CHOL, SEED)
    prob = pk.Problem(h, B, N_ORB // 2, N_ORB // 2, e0)
    sol = pk.Solver(prob, M=M, tol=1e-8, precision=args.precision)
    t_setup = time.time()
    for k in range(MID):
        sol.step(k, 0)
        print(f"# setup step {k} done", file=sys.stderr, flush=True)
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
    d = {k: s1[k] - s0[k] for k in s1}
    sig_flops = d["sigma_a_flops"] + d["sigma_b_flops"]
    tot_flops = sig_flops + d["env_flops"]
    ms_per_step = 1e3 * wall / args.steps
    nmv = max(d["matvecs"], 1)
    # dominant kernel: the long-K block GEMM of sigma (phase B); HIP-event time per launch of
    # the GEMM kernel alone (events on the solver stream around that launch)
    b_launch_ms = d["sigma_b_gemm_ms"] / nmv
    b_achieved = (d["sigma_b_flops"] / nmv) / (b_launch_ms * 1e-3) / 1e12 if b_launch_ms > 0 else 0.0
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
        "matvecs_per_step": nmv / args.steps,

        "breakdown_ms_per_step": {"sigma": (d["sigma_a_ms"] + d["sigma_b_ms"]) / args.steps,
                                  "env": d["env_ms"] / args.steps, "svd": d["svd_ms"] / args.steps,
                                  "prepare_wall": d["prepare_ms"] / args.steps,
                                  "plan_resolve_wall": d["resolve_ms"] / args.steps,
                                  "davidson_wall": d["davidson_ms"] / args.steps},
        "setup_s": t_setup,
        "energy_last": energies[-1] if energies else None,
        "plan_reuse_per_step": (d["plan_hits"]) / args.steps,
        "roofline": {"bound": "mfma", "kernel": "gemm_f64_w32<1, 4> (sigma phase B, timed launches)",
                     "achieved": b_achieved, "peak": PEAK_FP64, "unit": "TFLOP/s",
                     "frac": b_achieved / PEAK_FP64, "traffic": TRAFFIC,
                     "launch_ms": b_launch_ms, "flops_per_launch": d["sigma_b_flops"] / nmv},
    }
    if not args.no_sweep:
        # one full sweep (2(L-1) two-site steps) timed end to end; the centre first
        # walks back to site 0 with right-to-left steps (untimed)
        centre = MID + 1 if direction == 1 else MID
        for k in range(centre - 1, -1, -1):
            sol.step(k, 1)
        print("# centre at site 0", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        s2 = sol.stats()
        t0 = time.time()
        e, tau, ok = sol.sweep(1)
        torch.cuda.synchronize()
        sweep_s = time.time() - t0
        s3 = sol.stats()
        out["sweep"] = {"seconds": sweep_s, "steps": 2 * (N_ORB - 1), "energy": float(e[0]), "tau_max": tau,
                        "converged": bool(ok), "matvecs": s3["matvecs"] - s2["matvecs"],
                        "plan_reuse": s3["plan_hits"] - s2["plan_hits"],
                        "sigma_s": (s3["sigma_a_ms"] + s3["sigma_b_ms"] - s2["sigma_a_ms"] - s2["sigma_b_ms"]) / 1e3,
                        "tflops": (s3["sigma_a_flops"] + s3["sigma_b_flops"] + s3["env_flops"] - s2["sigma_a_flops"]
                                   - s2["sigma_b_flops"] - s2["env_flops"]) / sweep_s / 1e12}
        print(f"# sweep {sweep_s:.1f} s E={e[0]:.10f}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(pk, torch)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
