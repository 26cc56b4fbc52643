"""Write reference velocities of whole runs of the benchmark workloads (oracle only).

For each case below the FP64 oracle starts one sample of a workload from its
initial equilibrium (the workload's seed, flow parameters and Y of that
sample) and advances it by the number of steps the sample takes in the
workload's run. Stored per case:
  * the velocity u = j / rho at a regular subgrid of 16^3 nodes (every
    n/16-th node per axis, starting at node n/32 - 1, so no node sits on a
    symmetry plane of the Taylor-Green field), [3][16^3], x fastest;
  * the kinetic energy of the whole field, mean |u|^2 / 2;
  * the root mean square of |u| over the whole field and over the subgrid.

Cases (workload, sample, steps):
  * rtgv64x64_f32: samples 0, 21, 42, 63 of the 64 x 64^3 ensemble after
    1000 steps (the ensemble's 500-step run, continued to 1000);
  * mixed48_f32: samples 0 and 31 (64^3, 63 steps: ticks 0, 16, ..., 992),
    32 and 43 (128^3, 250 steps), 44 (256^3, 1000 steps) of the 1000-tick
    mixed-resolution run;
  * adjoint128x8_f32: samples 0 and 7 of the 8 x 128^3 forward run, 1000
    steps.

Usage: python tests/golden/make_velocity_reference.py [workload ...] [--threads T]
Output: tests/golden/velocity_<workload>.npz (numpy arrays only; no pickles).
"""
import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import mc_inputs  # noqa: E402
import oracle  # noqa: E402

SUB = 16

CASES = {
    "rtgv64x64_f32": [(0, 1000), (21, 1000), (42, 1000), (63, 1000)],
    "mixed48_f32": [(0, 63), (31, 63), (32, 250), (43, 250), (44, 1000)],
    "adjoint128x8_f32": [(0, 1000), (7, 1000)],
}


def subgrid_cells(n):
    """Cell indices (z*n + y)*n + x of the 16^3 subgrid, x fastest."""
    stride = n // SUB
    idx = np.arange(SUB) * stride + max(stride // 2 - 1, 0)
    z, y, x = np.meshgrid(idx, idx, idx, indexing="ij")
    return ((z * n + y) * n + x).reshape(-1).astype(np.int64)


def group_of(wl, sample):
    first = 0
    for g in wl.groups:
        if sample < first + g.count:
            return g
        first += g.count
    raise IndexError(sample)


def run_case(wl, y, sample, steps, threads):
    g = group_of(wl, sample)
    n = g.n
    om = oracle.omega_shear(oracle.lattice_viscosity(n, g.u0, g.re))
    t0 = time.time()
    f = oracle.init_populations(n, g.u0, g.amp, y[sample], g.project, wl.lattice)
    done = 0
    chunk = 50 if n <= 128 else 10
    while done < steps:
        k = min(chunk, steps - done)
        oracle.run(f, n, k, om, threads=threads)
        done += k
        print(f"  {wl.name} sample {sample} ({n}^3): {done}/{steps} steps, {time.time() - t0:.0f} s", flush=True)
    _, u = oracle.moments(f, n)
    del f
    u = u.reshape(3, -1)
    cells = subgrid_cells(n)
    usub = np.ascontiguousarray(u[:, cells])
    ke = float(oracle.kinetic_energy(u))
    rms = float(np.sqrt(np.mean(np.sum(u * u, axis=0))))
    rms_sub = float(np.sqrt(np.mean(np.sum(usub * usub, axis=0))))
    return dict(n=n, u0=g.u0, re=g.re, amp=g.amp, project=int(g.project), steps=steps, sample=sample,
                cells=cells, u=usub, ke=ke, rms=rms, rms_sub=rms_sub)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workloads", nargs="*", default=list(CASES))
    ap.add_argument("--threads", type=int, default=0)
    args = ap.parse_args()
    for name in args.workloads:
        wl = mc_inputs.WORKLOADS[name]
        y = mc_inputs.draw_y(wl.seed, wl.m)
        rows = [run_case(wl, y, s, steps, args.threads) for s, steps in CASES[name]]
        out = {
            "workload": np.array(name),
            "seed": np.int64(wl.seed),
            "m": np.int64(wl.m),
            "lattice": np.int64(wl.lattice),
            "y": y,
            "samples": np.array([r["sample"] for r in rows], dtype=np.int64),
            "steps": np.array([r["steps"] for r in rows], dtype=np.int64),
            "n": np.array([r["n"] for r in rows], dtype=np.int64),
            "ke": np.array([r["ke"] for r in rows]),
            "rms": np.array([r["rms"] for r in rows]),
            "rms_sub": np.array([r["rms_sub"] for r in rows]),
            "source": np.array("FP64 oracle (two-lattice pull, moment-space KBC), whole runs from the initial "
                               "equilibrium; u on the 16^3 subgrid"),
        }
        for k, r in enumerate(rows):
            out[f"cells_{k}"] = r["cells"]
            out[f"u_{k}"] = r["u"]
        path = os.path.join(HERE, f"velocity_{name}.npz")
        np.savez_compressed(path, **out)
        print(path, flush=True)


if __name__ == "__main__":
    main()
