"""The flexible-Prandtl collision (App. E, eq. Shakhov, with the term
shapes of reading D-Pr) on the GPU, through the C ABI (lbm_config.prandtl):
parity with the oracle's runs at the same Prandtl number on the same seeded
inputs (tolerances and metrics of test_gpu_parity.py), exact conservation
with one fixed lattice, graph replays equal to plain steps, and the
configurations the library refuses for it."""
import numpy as np
import pytest

import workloads as W
from test_gpu_parity import (TOL, check, gpu_run, lbm,  # noqa: F401
                             oracle_run, shift_disagreement)

pytestmark = pytest.mark.gpu


def _nosensor(wl, nu):
    wl.sensor = 0
    wl.nu = nu
    return wl


CASES = {
    "sod_256x1": (lambda: W.config0(), 200),
    "advected_sod_2048x4": (lambda: W.config1(2048, 4, 100), 100),
    "vortex_100": (lambda: W.isentropic_vortex(100, steps=60), 60),
    "quadrant_100": (lambda: W.four_quadrant(100, 40), 40),
    "quadrant_100_nosensor": (lambda: _nosensor(W.four_quadrant(100, 40), 3e-3), 40),
}


@pytest.mark.parametrize("Pr", [0.71, 2.0])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(CASES))
def test_parity_prandtl(lbm, orc, name, precision, Pr):
    make, steps = CASES[name]
    wl = make()
    print(f"case {name} Pr={Pr} {precision} {wl.nx}x{wl.ny} steps {steps}", flush=True)
    _, ref = oracle_run(orc, wl, steps, prandtl=Pr)
    sim, got = gpu_run(lbm, wl, steps, precision, prandtl=Pr)
    check(orc, got, ref, TOL[precision], f"{name}/Pr{Pr}/{precision}")
    shift_disagreement(got, ref)
    sim.close()


def test_conservation_with_one_lattice(lbm):
    wl = W.smooth_random(64, 48, seed=3, amp=(0.1, 0.3, 0.3, 0.15),
                         base=(1.0, 1.2, -0.3, 0.8), shift_mode=1, fixed_U=(1, 0), nu=5e-3)
    sim = lbm.Sim.from_workload(wl, precision="fp64", prandtl=0.71)
    c0 = np.array(sim.diag()["conserved"])
    sim.step(50)
    c1 = np.array(sim.diag()["conserved"])
    scale = np.array([c0[0], 3 * c0[0], 3 * c0[0], c0[3]])
    assert np.all(np.abs(c1 - c0) <= 64 * np.finfo(float).eps * 50 * scale), (c1 - c0) / scale
    sim.close()


def test_graph_replays_and_refusals(lbm):
    wl = W.four_quadrant(64, 20)
    a = lbm.Sim.from_workload(wl, precision="fp32", prandtl=0.71)
    b = lbm.Sim.from_workload(wl, precision="fp32", prandtl=0.71, schedule="auto")
    assert b.schedule == a.schedule and a.schedule["step_block"] == 64
    a.step(20)
    b.step_graph(20, chunk=10)
    ma = {k: v.cpu().numpy() for k, v in a.macros().items()}
    mb = {k: v.cpu().numpy() for k, v in b.macros().items()}
    for k in ("rho", "ux", "uy", "T", "Ux", "Uy"):
        assert np.array_equal(ma[k], mb[k]), k
    for bad in (dict(step_block=128), dict(tiles_per_block=2)):
        with pytest.raises(lbm.LBMError) as e:
            a.schedule = bad
        assert e.value.status == lbm.ERR_ARG
    with pytest.raises(lbm.LBMError) as e:
        lbm.step_batched([a, b], [2, 2])
    assert e.value.status == lbm.ERR_ARG
    for bad in (dict(constraints=4), dict(constraints=13),       # the latter: FP32
                dict(shift_mode=3, halfwidth=0.75), dict(prandtl=-1.0)):
        kw = dict(precision="fp32", prandtl=0.71)
        kw.update(bad)
        with pytest.raises(ValueError):
            lbm.Sim.from_workload(wl, **kw)
    # Pr = 1 is the BGK collision, bit for bit
    c = lbm.Sim.from_workload(wl, precision="fp32", prandtl=1.0)
    d = lbm.Sim.from_workload(wl, precision="fp32")
    c.step(5)
    d.step(5)
    assert np.array_equal(c.macros()["T"].cpu().numpy(), d.macros()["T"].cpu().numpy())
    for s in (a, b, c, d):
        s.close()
