"""Write FCI reference energies for the synthetic active spaces with the CPU oracle.

Run from the repository root:  python tests/golden/make_golden.py [names...]
Calls only ``synth`` (inputs) and ``oracle`` (the determinant FCI).  The output
``fci_energies.json`` is read by the GPU tests, which compare the DMRG energies
of the HIP path against it.
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import fci  # noqa: E402

CASES = {
    # name: (n, n_alpha, n_beta, n_chol, seed, nroots)
    "cas8_nq32_s0": (8, 4, 4, 32, 0, 3),
    "cas10_nq48_s0": (10, 5, 5, 48, 0, 2),
    "cas12_nq64_s0": (12, 6, 6, 64, 0, 3),
    "cas6_nq12_s3": (6, 3, 3, 12, 3, 3),
}

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fci_energies.json")


def main(names):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        n, na, nb, nq, seed, nroots = CASES[name]
        h, B, e0 = synth.make_hamiltonian(n, nq, seed)
        t = time.time()
        w, vs, space = fci.solve(n, na, nb, h, B, nroots=nroots, e_core=e0, tol=1e-8)
        s2 = [fci.s_squared_sparse(space, c) for c in vs]
        data[name] = {"n": n, "n_alpha": na, "n_beta": nb, "n_chol": nq, "seed": seed,
                      "energies": [float(x) for x in w], "s2": s2, "n_det": space.size,
                      "oracle_seconds": round(time.time() - t, 2)}
        print(name, data[name], flush=True)
        json.dump(data, open(OUT, "w"), indent=1)


if __name__ == "__main__":
    main(sys.argv[1:] or list(CASES))
