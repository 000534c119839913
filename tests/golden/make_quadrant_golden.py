"""Writes quadrant_<L>_<steps>.npz: sampled rows of the oracle's run of the
four-quadrant Riemann draw (the 4096^2, 1000-step configuration: seeded
quadrant states, Mach up to 3, nu = 1e-3, Knudsen sensor on) on an L^2 copy
of it, computed with the CPU oracle only.  Run from the repository root:

    python tests/golden/make_quadrant_golden.py [L steps]

Default: L = 512 and 125 steps, the copy in which the waves from the
quadrant lines cross the same fraction of the domain as in 1000 steps at
4096^2 (steps scaled with L).  Stored: the rows listed in `rows` of rho, ux,
uy, T and the lattice tags, the oracle's counters, the steps and the recipe.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402


def rows_of(L):
    """Eight rows: through the quadrant lines (L/2 and the seam at 0) and
    evenly spread others."""
    return np.unique(np.array([0, L // 8, L // 4, 3 * L // 8, L // 2, 5 * L // 8,
                               3 * L // 4, L - 1]))


def path_of(L, steps):
    return os.path.join(HERE, f"quadrant_{L}_{steps}.npz")


def make(L, steps):
    wl = W.config3(L, steps)
    t0 = time.time()
    s = oracle.Sim.from_workload(wl)
    done = 0
    while done < steps:
        n = min(25, steps - done)
        s.step(n)
        done += n
        print(f"quadrant {L}^2: {done}/{steps} steps, {time.time() - t0:.0f} s", flush=True)
    m = s.macros()
    st = s.stats()
    rows = rows_of(L)
    np.savez_compressed(
        path_of(L, steps), rows=rows, steps=np.int64(steps), L=np.int64(L),
        rho=m["rho"][rows], ux=m["ux"][rows], uy=m["uy"][rows], T=m["T"][rows],
        Ucx=m["Ucx"][rows].astype(np.int8), Ucy=m["Ucy"][rows].astype(np.int8),
        newton_calls=np.int64(st["newton_calls"]), newton_iters=np.int64(st["newton_iters"]),
        mismatched_links=np.int64(st["mismatched_links"]),
        recipe=np.array(f"workloads.config3({L}, {steps}): nu={wl.nu}, sensor={wl.sensor}"))


if __name__ == "__main__":
    if len(sys.argv) == 3:
        make(int(sys.argv[1]), int(sys.argv[2]))
    else:
        make(512, 125)
