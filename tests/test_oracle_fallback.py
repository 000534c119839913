"""The fallback equilibrium (lbm_config.fallback / orc_params.fallback): where
a state's 8-moment equilibrium, eq. (feqNum_8Mom), has no solution, that
solve takes the four-constraint equilibrium of eq. (feqNum_4Mom) instead.
The paper leaves the case open; these pin the oracle's reading of it.

- A uniform state whose velocity relative to a fixed lattice has no
  8-moment equilibrium is a fixed point of the fallback run: every node
  holds rho w4 (the four-constraint weights of the same state, solved
  directly) and (2 Cv - 2) T rho w4, and every solve is counted.
- Without the fallback the same state stops the run with ERR_NEWTON.
- On a quadrant draw that fails mid-run, the fallback run is bitwise the
  plain run up to the failure (it changes nothing where the 8-moment solve
  succeeds) and then runs on."""
import numpy as np
import pytest

import oracle
import workloads as W

# u' with no 8-moment solution on D2Q21 (the oracle's Newton fails from the
# Maxwellian) while the four-constraint one exists
UNSOLVABLE = (1.0, 1.58, -0.28, 1.38)


def test_state_has_no_8_moment_equilibrium():
    _, _, _, rc8 = oracle.equilibrium(*UNSOLVABLE[1:])
    w4, _, _, rc4 = oracle.equilibrium(*UNSOLVABLE[1:], constraints=4)
    assert rc8 == oracle.ERR_NEWTON and rc4 == oracle.OK
    cx, cy = (np.array(v, dtype=float) for v in zip(*oracle.velocities()))
    ux, uy, T = UNSOLVABLE[1:]
    # the four constraints hold: mass, momentum, energy (2E = |u|^2 + 2T)
    np.testing.assert_allclose([w4.sum(), (w4 * cx).sum(), (w4 * cy).sum(),
                                (w4 * (cx * cx + cy * cy)).sum()],
                               [1.0, ux, uy, ux * ux + uy * uy + 2 * T], rtol=0, atol=1e-13)


def test_uniform_unsolvable_state_is_a_fixed_point_of_the_fallback():
    rho, ux, uy, T = UNSOLVABLE
    wl = W.uniform(6, 4, rho, ux, uy, T, nu=1e-3, shift_mode=1, fixed_U=(0, 0))
    with pytest.raises(oracle.OracleError) as e:
        oracle.Sim.from_workload(wl)
    assert e.value.rc == oracle.ERR_NEWTON
    wl.fallback = 1
    s = oracle.Sim.from_workload(wl)
    steps = 5
    s.step(steps)
    w4, _, _, _ = oracle.equilibrium(ux, uy, T, constraints=4)
    f, g = s.populations()
    cv = 1.0 / (wl.gamma - 1.0)
    np.testing.assert_allclose(f, (rho * w4)[:, None, None] * np.ones_like(f), rtol=1e-13, atol=0)
    np.testing.assert_allclose(g, ((2 * cv - 2) * T * rho * w4)[:, None, None] * np.ones_like(g),
                               rtol=1e-13, atol=0)
    N = wl.nx * wl.ny
    # initial condition, its collision, then one collision per step
    assert s.stats()["fallbacks"] == N * (steps + 2)


def test_fallback_run_equals_plain_run_until_the_failure():
    job = {j.job_id: j for j in W.serving_jobs(10000)}[9006]  # 70^2 quadrant draw
    wl = job.build()
    assert wl.fallback == 1
    wl.fallback = 0
    plain = oracle.Sim.from_workload(wl)
    done = 0
    with pytest.raises(oracle.OracleError) as e:
        while done < 60:
            plain.step(1)
            done += 1
    assert e.value.rc == oracle.ERR_NEWTON and done >= 5
    wl.fallback = 1
    a = oracle.Sim.from_workload(wl)
    b = oracle.Sim.from_workload(wl)
    a.step(done)  # the last step the plain run completed
    ref = oracle.Sim.from_workload(_plain(wl))
    ref.step(done)
    for k in ("rho", "ux", "uy", "T"):
        assert np.array_equal(a.macros()[k], ref.macros()[k]), k
    assert a.stats()["fallbacks"] == 0
    b.step(done + 30)
    st = b.stats()
    assert st["fallbacks"] > 0 and st["steps"] == done + 30
    m = b.macros()
    assert np.all(m["rho"] > 0) and np.all(m["T"] > 0)


def _plain(wl):
    import copy
    w = copy.copy(wl)
    w.fallback = 0
    return w
