"""Writes vortex_<L>_<steps>.npz: sampled rows of the oracle's isentropic
vortex (the 1024^2, 5000-step configuration of Sec. IV-style high-Mach
tests: Mach 3 diagonal advection, strength 5, density noise 1e-4, tau =
1/2 + 1e-4 at the free-stream temperature, Knudsen sensor on), computed
with the CPU oracle only.  Run from the repository root:

    python tests/golden/make_vortex_golden.py [L steps]

Default: the full configuration, L = 1024 and 5000 steps (about two hours
of CPU on eight threads), and its quarter-size copy, L = 256 and 1250
steps, which makes the same number of vortex transits (the free stream
moves 2.1 nodes per step along each axis).  Stored per file: the rows
listed in `rows` of rho, ux, uy, T and the lattice tags Ucx, Ucy, the
oracle's Newton and rebuild counters, the steps and the field recipe.
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
    """Eight rows: through the vortex's start and end positions, the seam,
    and evenly spread others."""
    return np.unique(np.array([0, L // 8, L // 4, 3 * L // 8, L // 2, 5 * L // 8,
                               3 * L // 4, L - 1]))


def path_of(L, steps):
    return os.path.join(HERE, f"vortex_{L}_{steps}.npz")


def make(L, steps):
    wl = W.config2(L, steps)
    t0 = time.time()
    s = oracle.Sim.from_workload(wl)
    done = 0
    while done < steps:
        n = min(250, steps - done)
        s.step(n)
        done += n
        print(f"vortex {L}^2: {done}/{steps} steps, {time.time() - t0:.0f} s", flush=True)
    m = s.macros()
    st = s.stats()
    rows = rows_of(L)
    np.savez_compressed(
        path_of(L, steps), rows=rows, steps=np.int64(steps), L=np.int64(L),
        rho=m["rho"][rows], ux=m["ux"][rows], uy=m["uy"][rows], T=m["T"][rows],
        Ucx=m["Ucx"][rows].astype(np.int8), Ucy=m["Ucy"][rows].astype(np.int8),
        newton_calls=np.int64(st["newton_calls"]), newton_iters=np.int64(st["newton_iters"]),
        mismatched_links=np.int64(st["mismatched_links"]),
        recipe=np.array(f"workloads.config2({L}, {steps}): nu={wl.nu}, sensor={wl.sensor}"))
    print(f"wrote {path_of(L, steps)} in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    if len(sys.argv) == 3:
        make(int(sys.argv[1]), int(sys.argv[2]))
    else:
        make(256, 1250)
        make(1024, 5000)
