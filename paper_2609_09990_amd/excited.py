"""Excited states by penalty deflation with a per-root <S^2> guard (Sec. II.F).

Roots are found one at a time: each is a DMRG run of the library on the same
problem holding every state found before it (accepted or not) as a deflated
lower state, so its Davidson operator is H_eff + sum_j w |phi_j><phi_j|.  The
solver fixes N and S_z but is not spin-adapted; the spin is imposed by
selection on <S^2> (a root whose <S^2> is not S(S+1) for the requested S is
kept deflated but not reported) and verified on every reported root.  This
module only sequences library calls; the solves, projections, overlaps and
<S^2> run in the library's kernels.
"""
from __future__ import annotations

import numpy as np

from ._lib import Solver


def excited_states(problem, n_roots, M=256, weight=10.0, spin=None, s2_tol=1e-3, ovl_tol=1e-4,
                   sweeps=4, max_sweeps=20, conv_tol=1e-10, max_roots=None, **solver_kw):
    """The n_roots lowest states of `problem` (of total spin `spin` if given).

    weight: penalty (Ha) on each lower state; it must exceed the gap from that
    state to the target.  When a run ends with |<Psi|Phi_j>| > ovl_tol (the
    penalty was too weak to keep Psi off a lower state) the weight is doubled
    and the run repeated, up to 4 times.
    Each run sweeps at least `sweeps` times, then until two sweeps agree to
    conv_tol (at most max_sweeps).  max_roots bounds the number of runs
    (default 4 n_roots).
    Returns a dict: energies, s2, per-run records (energy, s2, overlaps with
    the held states, accepted, sweeps, weight) and the MPS of the reported roots.
    """
    target = None if spin is None else spin * (spin + 1.0)
    max_roots = 4 * n_roots if max_roots is None else max_roots
    held, runs, found = [], [], []
    while len(found) < n_roots and len(runs) < max_roots:
        w = float(weight)
        for _attempt in range(5):
            sol = Solver(problem, M=M, **solver_kw)
            for mps in held:
                sol.deflate(mps, w)
            e_prev, n_sw = None, 0
            while n_sw < max_sweeps:
                e, tau, ok = sol.sweep(1)
                n_sw += 1
                if n_sw >= sweeps and e_prev is not None and abs(e[0] - e_prev) < conv_tol:
                    break
                e_prev = e[0]
            ovl = [sol.overlap(j) for j in range(len(held))]
            if not ovl or max(abs(o) for o in ovl) <= ovl_tol:
                break
            w *= 2.0
        energy = float(sol.energy()[0])
        s2 = float(sol.s_squared()[0])
        mps = sol.export_mps()
        accepted = target is None or abs(s2 - target) <= s2_tol
        runs.append({"energy": energy, "s2": s2, "overlaps": ovl, "accepted": accepted, "sweeps": n_sw,
                     "weight": w, "converged": bool(ok), "tau": tau})
        held.append(mps)
        if accepted:
            found.append((energy, s2, mps))
        del sol
    return {"energies": np.array([f[0] for f in found]), "s2": np.array([f[1] for f in found]),
            "mps": [f[2] for f in found], "runs": runs}
