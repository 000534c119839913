"""The paper's reference model (App. C: D2Q49 with the 13 constraints of
eqs. G0-G4yyaa) on the GPU, through the C ABI (constraints = 13): parity
with the oracle's reference model on the same seeded inputs, FP64, to
1e-12 (metrics of test_gpu_parity.py), bitwise agreement of graph replays
with plain steps, and the configurations the library refuses for it."""
import numpy as np
import pytest

import workloads as W
from test_gpu_parity import check, gpu_run, lbm, oracle_run, shift_disagreement  # noqa: F401

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _fixed(wl, U):
    wl.shift_mode = 1
    wl.fixed_U = U
    return wl


CASES = {
    "sod_256x1": (lambda: W.config0(), 100),
    "advected_sod_512x2": (lambda: W.config1(512, 2, 50), 50),
    "quadrant_40": (lambda: W.four_quadrant(40, 20), 20),
    "quadrant_40_nosensor": (lambda: _nosensor(W.four_quadrant(40, 20)), 20),
    "vortex_40": (lambda: W.isentropic_vortex(40, steps=20), 20),
    "table1_32": (lambda: W.riemann_table1(32, steps=12), 12),
    "static_sod_256x1": (lambda: W.sod_static_shift(256, 1, steps=32), 32),
    "ragged_13x7": (lambda: W.smooth_random(13, 7, seed=2, shift_mode=0, nu=2e-3,
                                            base=(1.0, 0.6, -0.4, 0.8),
                                            amp=(0.1, 0.4, 0.4, 0.1)), 20),
    "fixed_U1_24x20": (lambda: _fixed(W.smooth_random(24, 20, seed=3, nu=5e-3,
                                                      base=(1.0, 1.2, -0.3, 0.8),
                                                      amp=(0.1, 0.3, 0.3, 0.1)), (1, 0)), 15),
}


def _nosensor(wl):
    wl.sensor = 0
    wl.nu = 3e-3
    return wl


@pytest.mark.parametrize("name", list(CASES))
def test_parity_reference_model(lbm, orc, name):
    make, steps = CASES[name]
    wl = make()
    print(f"case {name} D2Q49/M13 fp64 {wl.nx}x{wl.ny} steps {steps}", flush=True)
    s, ref = oracle_run(orc, wl, steps, constraints=13)
    sim, got = gpu_run(lbm, wl, steps, "fp64", constraints=13, stats=True)
    check(orc, got, ref, TOL, f"{name}/M13")
    shift_disagreement(got, ref)
    d = sim.diag()
    assert d["mismatched_links"] == s.stats()["mismatched_links"]
    sim.close()


PRANDTL_CASES = {
    "quadrant_40": (lambda: W.four_quadrant(40, 20), 20),
    "vortex_40": (lambda: W.isentropic_vortex(40, steps=20), 20),
    "advected_sod_512x2": (lambda: W.config1(512, 2, 50), 50),
}


@pytest.mark.parametrize("name", list(PRANDTL_CASES))
def test_parity_reference_model_prandtl(lbm, orc, name):
    """The flexible-Prandtl collision (App. E) on the reference model."""
    make, steps = PRANDTL_CASES[name]
    wl = make()
    print(f"case {name} D2Q49/M13 Pr=0.71 fp64 {wl.nx}x{wl.ny} steps {steps}", flush=True)
    _, ref = oracle_run(orc, wl, steps, constraints=13, prandtl=0.71)
    sim, got = gpu_run(lbm, wl, steps, "fp64", constraints=13, prandtl=0.71)
    check(orc, got, ref, TOL, f"{name}/M13/Pr0.71")
    shift_disagreement(got, ref)
    sim.close()


def test_populations_and_conserved_sums(lbm, orc):
    wl = CASES["fixed_U1_24x20"][0]()
    s, _ = oracle_run(orc, wl, 15, constraints=13)
    sim, _ = gpu_run(lbm, wl, 15, "fp64", constraints=13)
    f, g = (x.cpu().numpy() for x in sim.populations())
    assert f.shape == (49, wl.ny, wl.nx)
    vg = [tuple(v) for v in lbm.velocities(13)]
    vo = [tuple(v) for v in orc.velocities(49)]
    assert sorted(vg) == sorted(vo)
    fo, go = s.populations()
    perm = [vo.index(v) for v in vg]
    assert np.max(np.abs(f - fo[perm])) < 1e-13 * np.abs(fo).max()
    assert np.max(np.abs(g - go[perm])) < 1e-13 * np.abs(go).max()
    c = np.array(sim.diag()["conserved"])
    co = s.conserved()
    assert np.max(np.abs(c - co) / np.abs(co).max()) < 1e-13
    sim.close()


def test_graph_replays_match_plain_steps(lbm):
    wl = W.four_quadrant(40, 20)
    a = lbm.Sim.from_workload(wl, precision="fp64", constraints=13)
    b = lbm.Sim.from_workload(wl, precision="fp64", constraints=13)
    a.step(20)
    b.step_graph(20, chunk=4)
    ma = {k: v.cpu().numpy() for k, v in a.macros().items()}
    mb = {k: v.cpu().numpy() for k, v in b.macros().items()}
    for k in ("rho", "ux", "uy", "T", "Ux", "Uy"):
        assert np.array_equal(ma[k], mb[k]), k
    a.close()
    b.close()


def test_refused_configurations(lbm):
    wl = W.four_quadrant(24, 4)
    with pytest.raises(ValueError):      # FP32 storage is not built for it
        lbm.Sim.from_workload(wl, precision="fp32", constraints=13)
    with pytest.raises(ValueError):      # nor the neighbourhood shift choice
        lbm.Sim.from_workload(wl, precision="fp64", constraints=13, shift_mode=3,
                              halfwidth=0.75)
    sim = lbm.Sim.from_workload(wl, precision="fp64", constraints=13, schedule="auto")
    assert sim.schedule["step_block"] == 64 and sim.schedule["tiles_per_block"] == 1
    for bad in (dict(step_block=128), dict(tiles_per_block=2)):
        with pytest.raises(lbm.LBMError) as e:
            sim.schedule = bad
        assert e.value.status == lbm.ERR_ARG
    sim.schedule = dict(xcd_remap=0, rebuild_blocks=5)
    sim.step(2)
    other = lbm.Sim.from_workload(wl, precision="fp64", constraints=13)
    with pytest.raises(lbm.LBMError) as e:
        lbm.step_batched([sim, other], [2, 2])
    assert e.value.status == lbm.ERR_ARG
    sim.close()
    other.close()
