"""Writes sensitivity.json: how far the oracle drifts from itself when its
input is perturbed by one unit in the last place, on the long-horizon
configurations.  This is the flow's own amplification of rounding
differences (shocks and the sensor at low viscosity), the floor for any two
FP64 implementations that round differently; computed with the CPU oracle
only.  Run from the repository root:

    python tests/golden/make_sensitivity.py [case ...]

Cases: the advected Sod tube (2048 x 4, 2000 steps, workloads.config1),
the quarter-size copy of the isentropic vortex (256^2, 1250 steps,
workloads.config2(256, 1250)) and the 512^2 copy of the four-quadrant draw
(125 steps, workloads.config3(512, 125)).  Per checkpoint: max and median over nodes
of the relative error of rho, T and u (u relative to the largest |u|),
between the run from the drawn fields and the run whose initial density is
moved up by one ulp at every node.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

CASES = {
    "advected_sod_2048x4": (lambda: W.config1(2048, 4, 2000),
                            [150, 300, 500, 750, 1000, 1500, 2000]),
    "vortex_256": (lambda: W.config2(256, 1250), [100, 250, 500, 750, 1000, 1250]),
    "quadrant_512": (lambda: W.config3(512, 125), [25, 50, 75, 100, 125]),
}


def node_errors(a, b):
    e = np.maximum.reduce([np.abs(a["rho"] - b["rho"]) / np.abs(b["rho"]),
                           np.abs(a["T"] - b["T"]) / np.abs(b["T"]),
                           np.hypot(a["ux"] - b["ux"], a["uy"] - b["uy"]) /
                           np.max(np.hypot(b["ux"], b["uy"]))])
    return float(e.max()), float(np.median(e))


def run(name):
    make, checkpoints = CASES[name]
    wl = make()
    base = oracle.Sim.from_workload(wl)
    wl2 = make()
    wl2.rho = np.nextafter(wl2.rho, np.inf)
    pert = oracle.Sim.from_workload(wl2)
    out, done = [], 0
    for n in checkpoints:
        base.step(n - done)
        pert.step(n - done)
        done = n
        mx, med = node_errors(pert.macros(), base.macros())
        out.append(dict(steps=n, max=mx, median=med))
        print(f"{name} step {n}: max {mx:.2e} median {med:.2e}", flush=True)
    return out


if __name__ == "__main__":
    # python tests/golden/make_sensitivity.py [case ...]: all cases, or the
    # named ones merged into the existing file
    path = os.path.join(HERE, "sensitivity.json")
    names = sys.argv[1:] or list(CASES)
    res = {}
    if sys.argv[1:] and os.path.exists(path):
        with open(path) as f:
            res = json.load(f)
    res.update({name: run(name) for name in names})
    res["_doc"] = ("oracle against itself with the initial density moved up by one ulp: "
                   "max and median over nodes of the relative error of rho, T and u")
    with open(path, "w") as f:
        json.dump(res, f, indent=1)
