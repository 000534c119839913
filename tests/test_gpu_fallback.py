"""The fallback equilibrium on the GPU, through the C ABI: where a state's
8-moment equilibrium has no solution, lbm_config.fallback = 1 takes the
four-constraint one for that solve (the oracle's reading, pinned in
test_oracle_fallback.py).  Parity with the oracle at the tolerances of
test_gpu_parity.py, equal fallback counts, and a serving draw that stops
without the fallback running to its last step with it."""
import numpy as np
import pytest

import workloads as W
from test_gpu_parity import TOL, check, gpu_run, lbm, oracle_run, orc  # noqa: F401
from test_oracle_fallback import UNSOLVABLE, _plain

pytestmark = pytest.mark.gpu


def _job(job_id):
    return {j.job_id: j for j in W.serving_jobs(10000)}[job_id]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_uniform_unsolvable_state(lbm, orc, precision):
    rho, ux, uy, T = UNSOLVABLE
    wl = W.uniform(40, 24, rho, ux, uy, T, nu=1e-3, shift_mode=1, fixed_U=(0, 0))
    wl.fallback = 1
    steps = 5
    print(f"uniform unsolvable state {precision}", flush=True)
    o, ref = oracle_run(orc, wl, steps)
    sim, got = gpu_run(lbm, wl, steps, precision)
    check(orc, got, ref, TOL[precision], f"uniform fallback/{precision}")
    assert sim.diag()["fallback_solves"] == o.stats()["fallbacks"] == 40 * 24 * (steps + 2)
    sim.close()


def test_without_fallback_the_state_stops_the_run(lbm):
    rho, ux, uy, T = UNSOLVABLE
    wl = W.uniform(40, 24, rho, ux, uy, T, nu=1e-3, shift_mode=1, fixed_U=(0, 0))
    with pytest.raises(RuntimeError):
        gpu_run(lbm, wl, 1, "fp64")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_failing_serving_draw(lbm, orc, precision):
    """Serving job 9006 (70^2 quadrant draw, 300 steps) stops at step 14
    with the paper's equilibrium alone; with the fallback both sides run on
    and agree, taking the same fallbacks."""
    wl = _job(9006).build()
    assert wl.fallback == 1
    steps = 45
    print(f"job 9006 {precision} {wl.nx}x{wl.ny} steps {steps}", flush=True)
    o, ref = oracle_run(orc, wl, steps)
    sim, got = gpu_run(lbm, wl, steps, precision)
    check(orc, got, ref, TOL[precision], f"job 9006 fallback/{precision}")
    fb = o.stats()["fallbacks"]
    assert fb > 0
    if precision == "fp64":
        assert sim.diag()["fallback_solves"] == fb
    sim.close()


def test_failing_serving_draw_runs_to_the_end(lbm):
    job = _job(9006)
    wl = job.build()
    sim = lbm.Sim.from_workload(wl, precision="fp32")
    sim.step(job.steps)
    d = sim.diag()
    assert d["status"] == 0 and d["steps_done"] == job.steps and d["fallback_solves"] > 0
    sim.close()
    plain = lbm.Sim.from_workload(_plain(wl), precision="fp32")
    with pytest.raises(RuntimeError):
        plain.step(job.steps)
    plain.close()
