"""The four-constraint equilibrium (mass, momentum, energy; Sec. "Reduced
models", eq. feqNum_4Mom) on the GPU, through the C ABI: parity with the
oracle's four-constraint runs on the same seeded inputs (tolerances and
metrics of test_gpu_parity.py), the schedules it is built for, and batching
rules."""
import numpy as np
import pytest

import workloads as W
from test_gpu_parity import (TOL, check, gpu_run, lbm,  # noqa: F401
                             oracle_run, shift_disagreement)

pytestmark = pytest.mark.gpu

CASES = {
    "sod_256x1": (lambda: W.config0(), 200),
    "advected_sod_2048x4": (lambda: W.config1(2048, 4, 100), 100),
    "vortex_100": (lambda: W.isentropic_vortex(100, steps=60), 60),
    "quadrant_100": (lambda: W.four_quadrant(100, 40), 40),
    "quadrant_100_nosensor": (lambda: _nosensor(W.four_quadrant(100, 40), 3e-3), 40),
    "entropy_spot_100": (lambda: W.entropy_spot(2.0, steps=100), 100),
}


def _nosensor(wl, nu):
    wl.sensor = 0
    wl.nu = nu
    return wl


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(CASES))
def test_parity_four_constraints(lbm, orc, name, precision):
    make, steps = CASES[name]
    wl = make()
    print(f"case {name} M=4 {precision} {wl.nx}x{wl.ny} steps {steps}", flush=True)
    _, ref = oracle_run(orc, wl, steps, constraints=4)
    _, got = gpu_run(lbm, wl, steps, precision, constraints=4)
    check(orc, got, ref, TOL[precision], f"{name}/M4/{precision}")
    shift_disagreement(got, ref)


def test_uniform_state_stays_uniform(lbm):
    wl = W.uniform(40, 24, 1.0, 2.3, -0.7, 0.8, shift_mode=0)
    sim, m0 = gpu_run(lbm, wl, 0, "fp64", constraints=4)
    sim.step(25)
    m1 = {k: v.cpu().numpy() for k, v in sim.macros().items()}
    for k in ("rho", "ux", "uy", "T"):
        assert np.max(np.abs(m1[k] - m0[k])) < 1e-14, k


def test_sets_give_different_flows(lbm):
    """The variant is really a different equilibrium: at finite relative
    velocity the two sets' results differ far above rounding."""
    wl = W.isentropic_vortex(64, steps=20)
    _, a = gpu_run(lbm, wl, 20, "fp64", constraints=4)
    _, b = gpu_run(lbm, wl, 20, "fp64")
    assert np.max(np.abs(a["rho"] - b["rho"])) > 1e-6


def test_schedules_and_batches(lbm):
    wl = W.four_quadrant(64, 10)
    sim, _ = gpu_run(lbm, wl, 0, "fp32", constraints=4)
    assert sim.schedule["step_block"] == 64
    auto = lbm.Sim.from_workload(wl, precision="fp32", constraints=4, schedule="auto")
    assert auto.schedule == sim.schedule
    auto.close()
    for bad in (dict(step_block=128), dict(tiles_per_block=2)):
        with pytest.raises(lbm.LBMError) as e:
            sim.schedule = bad
        assert e.value.status == lbm.ERR_ARG
    sim.schedule = dict(xcd_remap=0, rebuild_blocks=7)    # allowed
    # a batch shares one constraint set
    other = lbm.Sim.from_workload(wl, precision="fp32")
    with pytest.raises(lbm.LBMError) as e:
        lbm.step_batched([sim, other], [3, 3])
    assert e.value.status == lbm.ERR_ARG
    # batched four-constraint jobs give the same bits as alone
    specs = [W.JobSpec(j, "quadrant" if j % 2 else "vortex", n, 1.0 + 0.5 * j, 15, 0.0)
             for j, n in enumerate((40, 56))]
    alone = []
    for sp in specs:
        s, m = gpu_run(lbm, sp.build(), sp.steps, "fp32", constraints=4)
        alone.append(m)
        s.close()
    sims = [lbm.Sim.from_workload(sp.build(), precision="fp32", constraints=4) for sp in specs]
    lbm.step_batched(sims, [sp.steps for sp in specs])
    for s, a in zip(sims, alone):
        got = {k: v.cpu().numpy() for k, v in s.macros().items()}
        for k in ("rho", "ux", "uy", "T", "Ux", "Uy"):
            assert np.array_equal(got[k], a[k]), k
        s.close()
