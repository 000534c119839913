"""Pins of the oracle's time stepping (streaming, reconstruction, collision,
lattice selection) to invariants and exact solutions."""
import json
import math
import os

import numpy as np
import pytest

import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
EPS = np.finfo(np.float64).eps


def run(orc, wl, steps, **over):
    s = orc.Sim.from_workload(wl, **over)
    s.step(steps)
    return s


@pytest.mark.parametrize("U", [(0, 0), (1, 0), (1, -1), (2, 0)])
def test_uniform_state_is_a_fixed_point(orc, U):
    """Equilibrium is a fixed point of eq. (coll): a uniform state stays
    uniform under any admissible fixed lattice shift."""
    wl = W.uniform(12, 10, 0.9, 1.3, -0.4, 0.8, nu=2e-3, shift_mode=1, fixed_U=U)
    s = run(orc, wl, 8)
    m = s.macros()
    for k, ref in [("rho", 0.9), ("ux", 1.3), ("uy", -0.4), ("T", 0.8)]:
        assert np.max(np.abs(m[k] - ref)) < 2e-14, k


@pytest.mark.parametrize("case", GOLD["criterion_examples"]["cases"])
def test_criterion_examples(orc, case):
    """Eq. (criterion) and the three examples that follow it."""
    lo, hi, U = np.array(case["u_lo"]), np.array(case["u_hi"]), case["U"]
    for t in (1e-6, 0.3, 0.77, 1 - 1e-6):   # inside (lo, hi], off the rounding-level ties
        u = lo + t * (hi - lo)
        wl = W.uniform(4, 4, 1.0, u[0], u[1], 0.7, shift_mode=0)
        m = run(orc, wl, 1).macros()
        assert (m["Ucx"] == U[0]).all() and (m["Ucy"] == U[1]).all(), (u, U)


def test_criterion_boundaries(orc):
    for u, U in [(0.5, 0), (np.nextafter(0.5, 1.0), 1), (-0.5, -1), (1.5, 1),
                 (np.nextafter(1.5, 2.0), 2)]:
        wl = W.uniform(3, 3, 1.0, u, 0.0, 0.7, shift_mode=0)
        s = orc.Sim.from_workload(wl)
        assert (s.macros()["Ucx"] == U).all(), (u, U)


def test_hysteresis_keeps_previous_lattice(orc):
    """Overlapping ranges (Sec. III.A.2, and n0 = 0.51 of Fig. 7): with a
    half-width above 1/2 the previous shift is kept while
    U_prev - w < u <= U_prev + w; with 1/2 the rule is eq. (criterion)."""
    sel = orc.select
    assert sel(0.495, 1, 0.51) == 1 and sel(0.495, 1, 0.5) == 0
    assert sel(0.505, 0, 0.51) == 0 and sel(0.505, 0, 0.5) == 1
    assert sel(1.505, 1, 0.51) == 1 and sel(1.505, 1, 0.5) == 2
    assert sel(1.7, 0, 0.51) == 2 and sel(-1.2, 0, 0.51) == -1
    for u in np.linspace(-3.2, 3.2, 257):
        assert sel(u, 7, 0.5) == math.ceil(u - 0.5)


@pytest.mark.parametrize("sensor", [0, 1])
def test_conservation_without_interfaces(orc, sensor):
    """With one fixed lattice, streaming is a permutation and the DDF BGK
    collision with tau_f = tau_g conserves mass, momentum and total energy
    (eqs. coll, gEq, polyTemp): the sums drift only by rounding."""
    wl = W.smooth_random(24, 20, seed=3, amp=(0.1, 0.3, 0.3, 0.1),
                         base=(1.0, 1.2, -0.3, 0.8), shift_mode=1, fixed_U=(1, 0),
                         nu=5e-3)
    s = orc.Sim.from_workload(wl, sensor=sensor)
    c0 = s.conserved()
    s.step(20)
    c1 = s.conserved()
    scale = np.array([c0[0], c0[0] * 3, c0[0] * 3, c0[3]])
    assert np.all(np.abs(c1 - c0) <= 64 * EPS * 20 * scale), (c1 - c0) / scale


def test_galilean_integer_shift_is_exact(orc):
    """Run A: lattice U = (a, b) and velocity u.  Run B: lattice 0 and
    velocity u - U.  All arithmetic is in the lattice frame, so
    f_A(x, t) = f_B(x - U t, t) bit for bit (Sec. I, eq. discrete_norm_peculiar)."""
    U = (1, -1)
    base = W.smooth_random(16, 12, seed=5, amp=(0.1, 0.3, 0.3, 0.1),
                           base=(1.0, 1.1, -0.9, 0.8), dyadic_bits=30,
                           shift_mode=1, fixed_U=U, nu=3e-3)
    A = orc.Sim.from_workload(base)
    wlB = W.Workload("B", base.nx, base.ny, base.rho, base.ux - U[0], base.uy - U[1],
                     base.T, base.nu, 0, 1, (0, 0))
    B = orc.Sim.from_workload(wlB)
    k = 5
    A.step(k)
    B.step(k)
    fA, gA = A.populations()
    fB, gB = B.populations()
    sh = (U[1] * k, U[0] * k)            # (dy, dx): f_A(x) = f_B(x - U t)
    assert np.array_equal(fA, np.roll(fB, sh, axis=(1, 2)))
    assert np.array_equal(gA, np.roll(gB, sh, axis=(1, 2)))
    mA, mB = A.macros(), B.macros()
    assert np.array_equal(mA["ux"], np.roll(mB["ux"] + U[0], sh, axis=(0, 1)))
    assert np.array_equal(mA["T"], np.roll(mB["T"], sh, axis=(0, 1)))


def test_uniform_state_across_static_interface(orc):
    """A uniform flow admissible in two lattices, with lattice 1 on part of the
    domain: every link crossing the interface is rebuilt by eq. (GradGeneral)
    with zero gradients, i.e. as the equilibrium of the receiving lattice at
    the source's state, which is exactly what streaming would deliver."""
    nx, ny = 16, 6
    wl = W.uniform(nx, ny, 1.1, 0.45, 0.2, 0.75, nu=4e-3, shift_mode=2)
    x = np.arange(nx)[None, :].repeat(ny, 0)
    wl.static_U = ((x >= 8).astype(np.int32), np.zeros((ny, nx), np.int32))
    s = orc.Sim.from_workload(wl)
    s.step(6)
    m = s.macros()
    assert s.stats()["mismatched_links"] > 0
    for k, ref in [("rho", 1.1), ("ux", 0.45), ("uy", 0.2), ("T", 0.75)]:
        assert np.max(np.abs(m[k] - ref)) < 5e-14, k
    assert set(np.unique(m["Ucx"])) == {0, 1}


def test_grad_nonequilibrium_carries_no_mass(orc):
    """The Grad deviation of eq. (GradGeneral_f) has zero zeroth moment on the
    lattice: sum_i f_eq cbar cbar = T I holds exactly (second-order
    constraints) and sigma is traceless; sum_i f_eq cbar_a (|cbar|^2/(2T) - Cp)
    vanishes by the first- and trace-third-order constraints.  A wrong trace
    term, frame or sign in the stress breaks this."""
    p = orc.make_params(8, 8, nu=0.05)
    du = np.array([0.03, -0.02, 0.05, 0.01])
    dT = np.array([0.02, -0.04])
    for L in [(0, 0), (1, 0), (1, 1)]:
        rho, ux, uy, T = 1.2, L[0] + 0.3, L[1] - 0.2, 0.9
        f0, g0, rc0 = orc.grad_populations(orc.make_params(8, 8, nu=0.0), rho, ux, uy, T,
                                            du, dT, L, 0)
        f, g, rc = orc.grad_populations(p, rho, ux, uy, T, du, dT, L, 0)
        assert rc == 0 and rc0 == 0
        assert abs((f - f0).sum()) < 1e-14 * rho
        assert abs((g - g0).sum()) < 1e-14 * g0.sum()
        assert np.max(np.abs(f - f0)) > 1e-4        # the deviation itself is not zero


def test_grad_stress_sign(orc):
    """For a shear du_x/dy = a > 0, -sigma_xy = mu a (Sec. III.B.2): the
    xy momentum flux of the Grad deviation is negative and close to sigma_xy
    (the lattice reproduces the needed fourth moments only approximately)."""
    nu, a, rho, T = 0.05, 0.02, 1.0, 0.7
    p = orc.make_params(8, 8, nu=nu)
    v = orc.velocities().astype(float)
    f, g, rc = orc.grad_populations(p, rho, 0.1, 0.0, T, [0.0, a, 0.0, 0.0], [0.0, 0.0],
                                    (0, 0), 0)
    w, *_ = orc.equilibrium(0.1, 0.0, T)
    fneq = f - rho * w
    flux = (fneq * (v[:, 0] - 0.1) * v[:, 1]).sum()
    sxy = -rho * nu * a
    assert flux < 0
    assert abs(flux - sxy) < 0.35 * abs(sxy)


def test_init_without_viscosity_is_equilibrium(orc):
    """nu = 0 makes the Grad deviation vanish: the stored state is the
    equilibrium of the input fields, whose moments are the inputs."""
    wl = W.smooth_random(12, 10, seed=9, shift_mode=0, nu=0.0)
    s = orc.Sim.from_workload(wl)
    m = s.macros()
    assert np.max(np.abs(m["rho"] - wl.rho)) < 1e-14
    assert np.max(np.abs(m["ux"] - wl.ux)) < 1e-14
    assert np.max(np.abs(m["T"] - wl.T)) < 1e-14


def sod_l1(orc, nx, steps, **kw):
    from oracle import riemann
    wl = W.sod(nx, 1, **kw) if "shift_mode" not in kw or kw["shift_mode"] != 2 else None
    s = orc.Sim.from_workload(wl)
    s.step(steps)
    m = s.macros()
    rho, u, p = riemann.periodic_sod_profile(nx, steps, nx // 2, (1, 1), (0.125, 0.1))
    return np.mean(np.abs(m["rho"][0] - rho)), np.mean(np.abs(m["ux"][0] - u)), s


def test_sod_matches_exact_riemann_solution(orc):
    """Sod tube of the 256 x 1 configuration, compared with the exact
    solution at step 32, before the waves of the two periodic Riemann
    problems meet (they meet at step 36.5).  Thresholds frozen from the
    oracle's first run (L1 rho 9.2e-3, u 1.43e-2)."""
    l1r, l1u, _ = sod_l1(orc, 256, 32)
    assert l1r < 1.0e-2 and l1u < 1.6e-2


@pytest.mark.slow
def test_sod_converges_under_refinement(orc):
    """Doubling resolution (and steps) reduces the L1 error."""
    errs = [sod_l1(orc, nx, t)[0] for nx, t in [(256, 32), (512, 64), (1024, 128)]]
    assert errs[1] < 0.7 * errs[0] and errs[2] < 0.7 * errs[1], errs


def test_sod_static_shift_like_unshifted(orc):
    """The paper's 'static' configuration (U_x = 1 on [L/2, 3L/4)): shock and
    contact travel through the lattice interface; the L1 error stays close to
    the unshifted run's (Sec. IV.C.1)."""
    from oracle import riemann
    base, _, _ = sod_l1(orc, 256, 32)
    wl = W.sod_static_shift(256, 1, steps=32)
    s = orc.Sim.from_workload(wl)
    s.step(32)
    m = s.macros()
    rho, u, p = riemann.periodic_sod_profile(256, 32, 128, (1, 1), (0.125, 0.1))
    l1 = np.mean(np.abs(m["rho"][0] - rho))
    assert s.stats()["mismatched_links"] > 0
    assert l1 < 1.3 * base, (l1, base)


def test_riemann2d_diagonal_symmetry(orc):
    """Table 1 states are symmetric about x = y (Sec. IV.C.2): rho is mirror
    symmetric and u_x, u_y swap, with adaptive lattices on both sides."""
    wl = W.riemann_table1(32, steps=12)
    s = orc.Sim.from_workload(wl)
    s.step(12)
    m = s.macros()
    assert s.stats()["mismatched_links"] > 0
    assert np.max(np.abs(m["rho"] - m["rho"].T)) < 1e-12
    assert np.max(np.abs(m["ux"] - m["uy"].T)) < 1e-12
    assert np.array_equal(m["Ucx"], m["Ucy"].T)


def test_shear_wave_dissipation_below_paper_levels(orc):
    """Sec. IV.B.1: inviscid shear wave on 100 x 1 at u0 = 2, 2.5, 3, compared
    at t = 15 t_c with the initial amplitude.  The paper prints 0.3/0.9/0.7 %;
    those depend on its (unprinted) velocity table, so this pins only the
    claim that all stay below 1 %."""
    g = GOLD["shear_wave_nu_num_percent"]
    for u0, steps, paper in zip(g["u0"], g["steps"], g["value"]):
        nx = 100
        x = np.arange(nx)[None, :]
        wl = W.Workload("shear", nx, 1, np.ones((1, nx)), np.full((1, nx), u0),
                        1e-3 * np.sin(2 * math.pi * x / nx), np.full((1, nx), 0.7),
                        0.0, steps, 0, (0, 0), 0.51)
        s = run(orc, wl, steps)
        nun = abs(1e-3 - s.macros()["uy"].max()) / 1e-3 * 100
        assert nun < 1.0, (u0, nun, paper)


def test_failures_are_reported(orc):
    """A lattice far from the flow leaves the solver's envelope: the oracle
    reports the failure instead of producing numbers."""
    wl = W.uniform(4, 4, 1.0, 4.0, 0.0, 0.7, shift_mode=1, fixed_U=(0, 0))
    s = orc.Sim(4, 4, shift_mode=1)
    with pytest.raises(orc.OracleError) as e:
        s.init(*wl.fields())
    assert e.value.rc == orc.ERR_NEWTON
    wl = W.uniform(4, 4, 1.0, 0.1, 0.0, -0.5, shift_mode=1)
    with pytest.raises(orc.OracleError) as e:
        s.init(*wl.fields())
    assert e.value.rc == orc.ERR_NONPHYSICAL
    wl = W.uniform(4, 4, 1.0, 7.2, 0.0, 0.7, shift_mode=0)
    with pytest.raises(orc.OracleError) as e:
        s2 = orc.Sim(4, 4, shift_mode=0, max_abs_shift=6)
        s2.init(*wl.fields())
    assert e.value.rc == orc.ERR_NONPHYSICAL


def test_printed_heat_flux_terms_carry_a_fraction_of_q(orc):
    """Reading D-6 as printed: the heat-flux moment (1/2) sum xi (|xi|^2 f + g)
    of a Grad state with q = -rho Cp nu grad T.  The g term 2 q.c/(rho Cp)
    contributes exactly (2 Cv - 2) T^2 / Cp q (it uses only the enforced
    moment sum xi_x^2 f_eq = rho T), i.e. 0.42 q at T = 0.7 instead of the
    internal-energy share; the f term adds about -0.27 q on this lattice, so
    the state carries ~0.15 q in total.  The same term forms make up the
    flexible-Prandtl correction of App. E, which is why that collision is
    built on corrected shapes instead (test_oracle_prandtl.py)."""
    v = orc.velocities().astype(float)
    nu, rho, T, dT = 0.05, 1.0, 0.7, 0.01
    p = orc.make_params(8, 8, nu=nu)
    f, g, rc = orc.grad_populations(p, rho, 0.0, 0.0, T, [0, 0, 0, 0], [dT, 0.0], (0, 0), 0)
    assert rc == 0
    w, *_ = orc.equilibrium(0.0, 0.0, T)
    Cv, Cp = 2.5, 3.5
    feq = rho * w
    geq = (2 * Cv - 2) * T * feq
    q = -rho * Cp * nu * dT
    qg = 0.5 * ((g - geq) * v[:, 0]).sum()
    qf = 0.5 * ((f - feq) * v[:, 0] * (v ** 2).sum(1)).sum()
    assert qg / q == pytest.approx((2 * Cv - 2) * T * T / Cp, rel=1e-12)
    assert -0.3 < qf / q < -0.25
    assert 0.1 < (qf + qg) / q < 0.2


def test_neighbourhood_choice_without_overlap_is_the_criterion(orc):
    """With half-width 1/2 the ranges do not overlap, every axis has one
    admissible shift, and the neighbourhood choice is eq. (criterion)."""
    wl = W.four_quadrant(40, 12)
    a = orc.Sim.from_workload(wl, shift_mode=0, halfwidth=0.5)
    b = orc.Sim.from_workload(wl, shift_mode=3, halfwidth=0.5)
    a.step(12)
    b.step(12)
    ma, mb = a.macros(), b.macros()
    for k in ("rho", "ux", "uy", "T", "Ucx", "Ucy", "Unx", "Uny"):
        assert np.array_equal(ma[k], mb[k]), k


def test_neighbourhood_choice_reduces_interface_cells(orc):
    """Sec. III.A.2: with overlapping ranges the shift can be chosen by the
    neighbourhood to reduce the number of interface cells.  On the seeded
    quadrant flow with half-width 0.9 it leaves fewer nodes next to another
    lattice than the history choice, and rebuilds fewer links."""
    wl = W.four_quadrant(100, 60)

    def run(mode):
        s = orc.Sim.from_workload(wl, shift_mode=mode, halfwidth=0.9)
        s.step(60)
        m = s.macros()
        cx, cy = m["Ucx"], m["Ucy"]
        diff = np.zeros(cx.shape, bool)
        for ax in (0, 1):
            for sh in (1, -1):
                diff |= (cx != np.roll(cx, sh, ax)) | (cy != np.roll(cy, sh, ax))
        return int(diff.sum()), s.stats()["mismatched_links"]

    hist, nb = run(0), run(3)
    assert nb[0] < 0.9 * hist[0], (hist, nb)
    assert nb[1] < hist[1], (hist, nb)


def test_neighbourhood_choice_needs_overlap_below_one(orc):
    with pytest.raises(ValueError):
        orc.Sim(8, 8, shift_mode=3, halfwidth=1.0)


def test_sensor_alpha_reading(orc):
    """The kinetic sensor's relaxation-time factor (Sec. IV.A.2, eq.
    DeltaAvg; alpha itself is not printed, reading D-S): no dissipation is
    added up to the paper's threshold eps = 0.01; the levels 1.05, 1.35 and
    2 hold from 0.011, 0.11 and 1.1 on; alpha is continuous (Lipschitz,
    largest slope 50 per unit eps, on the first ramp) and non-decreasing,
    so that a rounding-level change of eps changes tau by a rounding-level
    amount."""
    a = orc.sensor_alpha
    for e in (0.0, 1e-9, 5e-3, 0.00999, 0.01):
        assert a(e) == 1.0
    assert 1.0 < a(0.0101) < 1.05
    for e, level in ((0.011, 1.05), (0.05, 1.05), (0.1, 1.05), (0.11, 1.35), (0.5, 1.35),
                     (1.0, 1.35), (1.1, 2.0), (50.0, 2.0)):
        assert abs(a(e) - level) < 1e-13, (e, a(e))
    xs = np.unique(np.concatenate([np.linspace(0.0, 3.0, 300001), np.geomspace(1e-4, 50.0, 4001),
                                   [0.01, 0.011, 0.1, 0.11, 1.0, 1.1]]))
    v = np.array([a(x) for x in xs])
    assert np.all(np.diff(v) >= 0.0)
    assert np.all(np.diff(v) <= 50.0 * np.diff(xs) * (1 + 1e-9) + 1e-14)
    assert v.max() == 2.0
    for knot in (0.01, 0.011, 0.1, 0.11, 1.0, 1.1):
        assert abs(a(knot * (1 + 1e-12)) - a(knot * (1 - 1e-12))) < 1e-10


def test_shear_wave_gap_reading(orc):
    """Reading D-L4 (Sec. IV.B.1).  At u0 = 2 and u0 = 3 the criterion picks
    U = u0, so both runs are the same flow at rest in its lattice (u' = 0):
    integer shifts are exact, so after the same number of steps the two
    transverse-velocity fields are equal up to the translation by the
    shift.  The peak loss of that one trajectory oscillates (an acoustic
    mode of the initial state) between about 0.01 % and 0.12 % over the
    first 1000 steps, so the printed 0.3 % (u0 = 2, 750 steps) and 0.7 %
    (u0 = 3, 500 steps) lie above anything this trajectory reaches at any
    time; with every admissible fixed lattice (u' = 0, +-1/2, +-1) the
    figures stay below 0.1 % as well."""
    nx = 100
    x = np.arange(nx)[None, :]

    def wave(u0):
        return W.Workload("shear", nx, 1, np.ones((1, nx)), np.full((1, nx), u0),
                          1e-3 * np.sin(2 * math.pi * x / nx), np.full((1, nx), 0.7),
                          0.0, 0, 0, (0, 0), 0.51)

    a = orc.Sim.from_workload(wave(2.0))
    b = orc.Sim.from_workload(wave(3.0))
    loss = []
    for k in range(30):
        a.step(25)
        b.step(25)
        ma, mb = a.macros(), b.macros()
        assert np.all(ma["Ucx"] == 2) and np.all(mb["Ucx"] == 3)
        t = 25 * (k + 1)                     # b has moved t cells further
        assert np.array_equal(np.roll(ma["uy"], t, axis=1), mb["uy"])
        loss.append(100 * (1.0 - ma["uy"].max() / 1e-3))
    g = GOLD["shear_wave_nu_num_percent"]
    paper = dict(zip(g["u0"], g["value"]))
    assert max(loss) < min(paper.values()) / 2
    assert min(loss) >= 0.0
