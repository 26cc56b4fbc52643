"""Write the reference gradient of the ensemble-mean kinetic energy (oracle only).

J = (1/M) sum_m KE_m(T) for M = 2 RTGV samples at 32^3 (U0 = 0.05, Re = 100,
amp = 0.05, projected perturbation, Y from SplitMix64 seed 2610), T = 1000
steps. dJ/dY_m = (1/M) dKE_m/dY_m by the complex step of the FP64 oracle
(h = 1e-30, exact to rounding). Output: gradient_rtgv32_T1000.json.

Usage: python tests/golden/make_gradient_reference.py [steps]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import mc_inputs  # noqa: E402
import oracle  # noqa: E402


def main():
    steps = int(sys.argv[1]) if len(sys.argv) > 1 else 1000
    n, u0, re, amp, project, seed, m = 32, 0.05, 100.0, 0.05, True, 2610, 2
    y = mc_inputs.draw_y(seed, m)
    out = {"n": n, "u0": u0, "re": re, "amp": amp, "project": project, "seed": seed, "m": m, "steps": steps,
           "y": y.tolist(), "ke": [], "dJdY": [],
           "source": "complex step (h = 1e-30) of the FP64 oracle; J = (1/M) sum_m KE_m(T)"}
    t0 = time.time()
    for s in range(m):
        ke = oracle.ke_after(n, u0, re, amp, y[s], project, steps)
        g = oracle.ke_gradient_complex_step(n, u0, re, amp, y[s], project, steps)
        out["ke"].append(ke)
        out["dJdY"].append((g / m).tolist())
        print(f"sample {s}: KE = {ke:.12e}, |dKE/dY| = {np.linalg.norm(g):.6e} ({time.time() - t0:.0f} s)",
              flush=True)
    path = os.path.join(HERE, f"gradient_rtgv32_T{steps}.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(path)


if __name__ == "__main__":
    main()
