"""The seeded input generators: shapes, determinism and the stated recipes."""
import math

import numpy as np

import workloads as W


def test_config_shapes():
    for wl, shape in [(W.config0(), (1, 256)), (W.config1(64, 4, 10), (4, 64)),
                      (W.config2(64, 10), (64, 64)), (W.config3(64, 10), (64, 64))]:
        for a in wl.fields():
            assert a.shape == shape and a.dtype == np.float64 and a.flags.c_contiguous
        assert np.all(wl.rho > 0) and np.all(wl.T > 0)


def test_sod_states():
    wl = W.config0()
    assert wl.rho[0, 0] == 1.0 and wl.rho[0, -1] == 0.125
    assert wl.T[0, 0] == 1.0 and abs(wl.T[0, -1] - 0.8) < 1e-15
    assert wl.shift_mode == 1 and wl.fixed_U == (0, 0) and wl.nu == 1e-3
    c1 = W.config1()
    assert abs(c1.ux[0, 0] - 2 * math.sqrt(1.4)) < 1e-15 and c1.shift_mode == 0


def test_vortex_recipe():
    wl = W.isentropic_vortex(256, noise=0.0)
    assert abs(wl.meta["u_inf"][0] - 2.1) < 1e-12           # Mach 3 on the diagonal
    du = np.hypot(wl.ux - 2.1, wl.uy - 2.1)
    assert abs(du.max() - 0.666) < 2e-3
    assert abs(wl.T.min() - 0.528) < 2e-3 and abs(wl.rho.min() - 0.494) < 2e-3
    assert abs(wl.nu - 7e-5) < 1e-18
    n = W.isentropic_vortex(256)
    rel = n.rho / wl.rho - 1
    assert 0.9e-4 < np.abs(rel).max() <= 1e-4 and np.array_equal(n.T, wl.T)
    assert np.array_equal(W.isentropic_vortex(256).rho, n.rho)  # seeded


def test_quadrant_draw_constraints():
    for sub in range(20):
        wl = W.four_quadrant(32, 10, sub=sub)
        Ts = [s[3] / s[0] for s in wl.meta["states"]]
        assert max(Ts) / min(Ts) <= 2 and min(Ts) >= 0.5 and max(Ts) <= 1.4
        assert 0 <= wl.meta["mach"] <= 3
        for r, ux, uy, p in wl.meta["states"]:
            assert 0.5 <= r <= 1.5 and 0.03 <= p <= 1.5
    a, b = W.four_quadrant(16, 1), W.four_quadrant(16, 1)
    assert np.array_equal(a.ux, b.ux)


def test_table1_is_diagonal_symmetric():
    wl = W.riemann_table1(40)
    assert np.array_equal(wl.rho, wl.rho.T) and np.array_equal(wl.ux, wl.uy.T)


def test_serving_mix_distribution():
    jobs = W.serving_jobs(4000)
    sides = np.array([j.side for j in jobs])
    steps = np.array([j.steps for j in jobs])
    mach = np.array([j.mach for j in jobs])
    assert sides.min() >= 64 and sides.max() <= 1024
    assert abs(np.median(np.log(sides)) - 0.5 * (math.log(64) + math.log(1024))) < 0.1
    assert steps.min() >= 100 and steps.max() <= 2000
    assert 0.5 <= mach.min() and mach.max() <= 3.0
    frac = np.mean([j.kind == "vortex" for j in jobs])
    assert 0.45 < frac < 0.55
    assert jobs[17].build().nx == jobs[17].side


def test_window_is_periodic_crop():
    wl = W.config3(32, 1)
    w = wl.window(1, 30, 3)
    assert w.nx == 7 and w.rho[3, 3] == wl.rho[30, 1] and w.rho[0, 0] == wl.rho[27, 30]
