"""Error of the FP32-storage form against the FP64 form, per benchmark
configuration, over the configurations' own horizons (the FP64 GPU form is
the oracle's to 1e-12 on every parity case, so it stands in for the oracle
at sizes the oracle cannot run).  Printed as a report; the asserted bounds
are the measured levels with a margin of about 2.5, so that a regression
shows.

FP32 rounding of the stored populations (~6e-8 per step) is amplified by
the flows themselves (shocks, and tau close to 1/2 in the vortex): the
same dynamics take a one-ulp FP64 perturbation of the oracle's input to
8e-7 over the advected Sod's 2000 steps (tests/golden/sensitivity.json).
So the error grows with the horizon: the 1e-5 max-norm bound holds over
the parity tests' horizons (<= 200 steps), not over thousands of steps,
where these are the form's stated errors."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

CASES = {
    # name: (workload, steps, bound on the max error, bound on the L1 error)
    "C0_sod_256x1": (lambda: W.config0(), 200, 5e-6, 8e-7),
    "C1_advected_sod_2048x4": (lambda: W.config1(2048, 4, 2000), 2000, 1.2e-2, 4e-4),
    "C2_vortex_1024": (lambda: W.config2(1024, 5000), 5000, 7e-3, 4e-4),
    "C3_quadrant_4096": (lambda: W.config3(4096, 1000), 1000, 2.4e-1, 7e-4),
}


@pytest.fixture(scope="module")
def lbm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2009_13426_amd as lbm
    return lbm


def run(lbm, wl, steps, precision):
    import torch
    sim = lbm.Sim.from_workload(wl, precision=precision)
    sim.step(steps)
    m = {k: v.cpu().numpy() for k, v in sim.macros().items()}
    sim.close()
    torch.cuda.empty_cache()
    return m


@pytest.mark.parametrize("name", list(CASES))
def test_fp32_error_against_fp64(lbm, name):
    make, steps, max_bound, l1_bound = CASES[name]
    wl = make()
    a = run(lbm, wl, steps, "fp32")
    b = run(lbm, wl, steps, "fp64")
    e = {}
    for k in ("rho", "T"):
        d = np.abs(a[k] - b[k])
        e[k] = (float(np.max(d / np.abs(b[k]))), float(d.sum() / np.abs(b[k]).sum()))
    du = np.hypot(a["ux"] - b["ux"], a["uy"] - b["uy"])
    um = np.hypot(b["ux"], b["uy"])
    e["u"] = (float(du.max() / um.max()), float(du.sum() / um.sum()))
    print(f"{name} ({steps} steps) FP32 vs FP64: " +
          ", ".join(f"{k} max {v[0]:.2e} L1 {v[1]:.2e}" for k, v in e.items()), flush=True)
    assert max(v[0] for v in e.values()) <= max_bound, e
    assert max(v[1] for v in e.values()) <= l1_bound, e
