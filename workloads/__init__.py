"""Seeded synthetic inputs for the adaptive D2Q21 compressible LBM.

This module only draws and lays out macroscopic initial fields (density,
velocity, temperature) and run parameters.  It contains none of the lattice
Boltzmann arithmetic: no equilibrium, no collision, no streaming.  Both the
CPU oracle and the HIP path receive their inputs from here, so it must stay
free of either side's code.

Every field is a C-contiguous float64 array of shape (ny, nx), node (x, y)
at index [y, x], periodic in both directions.  Temperature is T = p / rho
(lattice units, gas constant 1).  The flows follow the paper's validation
section (Sec. IV): the Sod tube (Sec. IV.C.1), the 2D Riemann problem of
Table 1 (Sec. IV.C.2), plus an isentropic vortex and seeded four-quadrant
Riemann draws shaped like those high-Mach test cases.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Tuple

import numpy as np

SEED_BASE = 2009134260
GAMMA = 1.4          # heat capacity ratio used by every test in Sec. IV
T0 = 0.7             # D2Q21 reference temperature (App. D, table of T0)
RHO0 = 1.0


def rng_for(config_index: int, extra: int = 0) -> np.random.Generator:
    """PCG64 stream for a given config (seed base + index, optional sub-stream)."""
    return np.random.Generator(np.random.PCG64([SEED_BASE + config_index, extra]))


@dataclasses.dataclass
class Workload:
    """A named initial state plus the run parameters that go with it."""
    name: str
    nx: int
    ny: int
    rho: np.ndarray
    ux: np.ndarray
    uy: np.ndarray
    T: np.ndarray
    nu: float
    steps: int
    shift_mode: int = 0          # 0 = adaptive criterion, 1 = fixed lattice
    fixed_U: Tuple[int, int] = (0, 0)
    halfwidth: float = 0.5
    gamma: float = GAMMA
    sensor: int = 0              # 1: Knudsen-number sensor on the relaxation time
    static_U: Tuple = None       # (Ux, Uy) int arrays for shift_mode 2
    fallback: int = 0            # 1: four-constraint equilibrium where the 8-moment one fails
    meta: Dict = dataclasses.field(default_factory=dict)

    @property
    def nodes(self) -> int:
        return self.nx * self.ny

    def fields(self):
        return self.rho, self.ux, self.uy, self.T

    def window(self, cx: int, cy: int, half: int) -> "Workload":
        """Periodic sub-block of side 2*half+1 centred on node (cx, cy).

        Used to evaluate a few nodes of a large run on a small periodic copy:
        values near the copy's centre are unaffected by its artificial seam
        for as many steps as the seam needs to reach the centre.
        """
        xs = (np.arange(cx - half, cx + half + 1) % self.nx)
        ys = (np.arange(cy - half, cy + half + 1) % self.ny)
        sub = lambda a: np.ascontiguousarray(a[np.ix_(ys, xs)])
        return dataclasses.replace(self, name=f"{self.name}@({cx},{cy})",
                                   nx=2 * half + 1, ny=2 * half + 1,
                                   rho=sub(self.rho), ux=sub(self.ux),
                                   uy=sub(self.uy), T=sub(self.T))


def _grid(nx: int, ny: int):
    x = np.arange(nx, dtype=np.float64)[None, :].repeat(ny, 0)
    y = np.arange(ny, dtype=np.float64)[:, None].repeat(nx, 1)
    return x, y


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- Sod tube
def sod(nx: int = 256, ny: int = 1, x0: int | None = None, u0: float = 0.0,
        left=(1.0, 1.0), right=(0.125, 0.1), nu: float = 1e-3,
        steps: int = 200, shift_mode: int = 1, fixed_U=(0, 0),
        halfwidth: float = 0.5, name: str = "sod", sensor: int = 1) -> Workload:
    """Two-state Riemann tube: (rho, p) = left for x < x0, right otherwise.

    Periodic, so a second discontinuity sits at the seam x = 0.  The
    Knudsen-number sensor is on by default, as in the paper's shock tests
    (Sec. IV.C).
    """
    x0 = nx // 2 if x0 is None else x0
    x, _ = _grid(nx, ny)
    L = x < x0
    rho = np.where(L, left[0], right[0])
    p = np.where(L, left[1], right[1])
    return Workload(name, nx, ny, _c(rho), _c(np.full_like(rho, u0)),
                    _c(np.zeros_like(rho)), _c(p / rho), nu, steps,
                    shift_mode, tuple(fixed_U), halfwidth, sensor=sensor,
                    meta=dict(x0=x0, left=left, right=right, u0=u0))


def sod_static_shift(nx: int = 256, ny: int = 1, steps: int = 32, nu: float = 1e-3,
                     Ux: int = 1) -> Workload:
    """The paper's 'static' Sod configuration (Sec. IV.C.1, Fig. 7): lattice
    shift U_x = Ux on L/2 <= x < 3L/4 and 0 elsewhere, fixed in time."""
    wl = sod(nx, ny, nu=nu, steps=steps, shift_mode=2, name=f"sod_static_{nx}x{ny}")
    x, _ = _grid(nx, ny)
    ux_map = np.where((x >= nx // 2) & (x < 3 * nx // 4), Ux, 0).astype(np.int32)
    wl.static_U = (ux_map, np.zeros_like(ux_map))
    return wl


def config0() -> Workload:
    """256x1 Sod tube, fixed lattice U = 0, nu = 1e-3, 200 steps."""
    return sod(256, 1, name="sod_256x1_fixedU0")


def config1(nx: int = 2048, ny: int = 4, steps: int = 2000,
            halfwidth: float = 0.6) -> Workload:
    """Sod states advected at Mach 2 of the left state, adaptive lattice with
    overlapping velocity ranges chosen by history (Sec. III.A.2): a node keeps
    its shift while |u - U| <= halfwidth.  With the plain criterion (0.5) the
    shocks from the two discontinuities meet near step 297 and a rebuilt link
    there needs |u'| > 2 in the receiver's lattice, outside the range the
    8-moment D2Q21 equilibrium can represent."""
    u0 = 2.0 * math.sqrt(GAMMA * 1.0)     # sound speed of the left (driver) state
    return sod(nx, ny, u0=u0, steps=steps, shift_mode=0, halfwidth=halfwidth,
               name=f"advected_sod_{nx}x{ny}")


# ------------------------------------------------------ isentropic vortex
def isentropic_vortex(L: int = 1024, mach: float = 3.0, beta: float = 5.0,
                      noise: float = 1e-4, steps: int = 5000,
                      nu: float | None = None, seed_index: int = 2,
                      T_inf: float = T0, rho_inf: float = RHO0,
                      name: str | None = None, sensor: int = 1) -> Workload:
    """Isentropic vortex of strength beta, radius L/10, advected diagonally.

    The free stream moves at `mach` times the free-stream sound speed along
    the diagonal; at Mach 3 and T_inf = 0.7 each component is exactly 2.1.
    Velocity is scaled by sqrt(T_inf), temperature drop by T_inf.  Density
    carries seeded uniform relative noise of amplitude `noise` at fixed u, T.
    At nu = 1e-4 T_inf (tau = 1/2 + 1e-4) this is the low-viscosity regime in
    which the paper turns the Knudsen-number sensor on (Sec. IV.A.2); it is on
    by default.
    """
    R = L / 10.0
    c_inf = math.sqrt(GAMMA * T_inf)
    comp = mach * c_inf / math.sqrt(2.0)
    x, y = _grid(L, L)
    dx = (x - L / 2 + L / 2) % L - L / 2          # nearest periodic image
    dy = (y - L / 2 + L / 2) % L - L / 2
    xb, yb = dx / R, dy / R
    r2 = xb * xb + yb * yb
    amp = beta / (2 * math.pi) * np.exp(0.5 * (1.0 - r2)) * math.sqrt(T_inf)
    ux = comp - amp * yb
    uy = comp + amp * xb
    T = T_inf * (1.0 - (GAMMA - 1) * beta ** 2 / (8 * GAMMA * math.pi ** 2)
                 * np.exp(1.0 - r2))
    rho = rho_inf * (T / T_inf) ** (1.0 / (GAMMA - 1))
    if noise:
        rng = rng_for(seed_index)
        rho = rho * (1.0 + noise * rng.uniform(-1.0, 1.0, size=rho.shape))
    nu = 1e-4 * T_inf if nu is None else nu
    return Workload(name or f"vortex_{L}x{L}_M{mach:g}", L, L, _c(rho), _c(ux),
                    _c(uy), _c(T), nu, steps, 0, (0, 0), 0.5, sensor=sensor,
                    meta=dict(R=R, beta=beta, u_inf=(comp, comp), mach=mach))


def config2(L: int = 1024, steps: int = 5000) -> Workload:
    return isentropic_vortex(L, steps=steps)


# ------------------------------------------------- four-quadrant Riemann
def quadrant_fields(L: int, states) -> Tuple[np.ndarray, ...]:
    """Lay out four (rho, ux, uy, p) states: [1] upper right, [2] upper left,
    [3] lower left, [4] lower right (the numbering of Table 1)."""
    x, y = _grid(L, L)
    right = x >= L // 2
    top = y >= L // 2
    q = np.where(top & right, 0, np.where(top & ~right, 1,
                 np.where(~top & ~right, 2, 3)))
    S = np.asarray(states, dtype=np.float64)     # (4, 4): rho, ux, uy, p
    rho, ux, uy, p = (S[q, k] for k in range(4))
    return _c(rho), _c(ux), _c(uy), _c(p / rho)


TABLE1 = [  # (rho, ux, uy, p) per quadrant, as printed in Table 1
    (0.513, 0.0, 0.0, 0.4),
    (1.0, 0.7276, 0.0, 1.0),
    (0.8, 0.0, 0.0, 1.0),
    (1.0, 0.0, 0.7276, 1.0),
]


def riemann_table1(L: int = 200, nu: float = 1e-3, steps: int = 100) -> Workload:
    rho, ux, uy, T = quadrant_fields(L, TABLE1)
    return Workload(f"riemann2d_table1_{L}", L, L, rho, ux, uy, T, nu, steps, sensor=1,
                    meta=dict(states=TABLE1))


# Viscosity of the seeded four-quadrant draws.  With the Knudsen-number
# sensor on (as in the paper's 2D Riemann runs, Sec. IV.C.2) nu = 1e-3 runs
# the seeded draw without equilibrium-solver failures; without the sensor it
# fails within 50 steps.
QUADRANT_NU = 1e-3


def initial_lattice(u: float) -> int:
    """Lattice shift of a velocity component at t = 0 (eq. criterion)."""
    return int(math.ceil(u - 0.5))


def links_within(states, max_speed: float) -> bool:
    """True if every quadrant's state, seen in every other quadrant's initial
    lattice, moves at most max_speed relative to that lattice: the states the
    first steps rebuild links at (a rebuilt link takes the source's state in
    the receiver's lattice)."""
    for a in states:
        for b in states:
            Ux, Uy = initial_lattice(b[1]), initial_lattice(b[2])
            if math.hypot(a[1] - Ux, a[2] - Uy) > max_speed:
                return False
    return True


def draw_quadrant_states(rng: np.random.Generator, mach_range=(0.0, 3.0),
                         mach: float | None = None, T_ref: float = T0,
                         max_link_speed: float | None = None):
    """Seeded four-quadrant draw: a common velocity (Mach in mach_range w.r.t.
    T_ref, random direction), then per quadrant rho ~ U[0.5, 1.5] and
    p ~ U[0.03, 1.5] redrawn until T = p / rho lies in [0.5, 1.4], plus a
    velocity perturbation of magnitude U[0, 0.75] in a random direction.
    Draws with T_max / T_min > 2 are rejected as a whole, and so are draws
    with a quadrant moving faster than max_link_speed relative to another
    quadrant's lattice (when given)."""
    c0 = math.sqrt(GAMMA * T_ref)
    while True:
        M = rng.uniform(*mach_range) if mach is None else mach
        th = rng.uniform(0.0, 2 * math.pi)
        U = M * c0 * np.array([math.cos(th), math.sin(th)])
        states = []
        for _ in range(4):
            while True:
                rho = rng.uniform(0.5, 1.5)
                p = rng.uniform(0.03, 1.5)
                if 0.5 <= p / rho <= 1.4:
                    break
            a = rng.uniform(0.0, 0.75)
            ph = rng.uniform(0.0, 2 * math.pi)
            states.append((rho, U[0] + a * math.cos(ph), U[1] + a * math.sin(ph), p))
        Ts = [s[3] / s[0] for s in states]
        if max(Ts) / min(Ts) <= 2.0 and (max_link_speed is None or
                                         links_within(states, max_link_speed)):
            return states, M


def four_quadrant(L: int = 4096, steps: int = 1000, seed_index: int = 3,
                  nu: float | None = None, sub: int = 0,
                  mach: float | None = None,
                  max_link_speed: float | None = None) -> Workload:
    rng = rng_for(seed_index, sub)
    states, M = draw_quadrant_states(rng, mach=mach, max_link_speed=max_link_speed)
    rho, ux, uy, T = quadrant_fields(L, states)
    return Workload(f"quadrant_{L}x{L}_s{seed_index}.{sub}", L, L, rho, ux, uy, T,
                    QUADRANT_NU if nu is None else nu, steps, sensor=1,
                    meta=dict(states=states, mach=M))


def config3(L: int = 4096, steps: int = 1000) -> Workload:
    return four_quadrant(L, steps)


# ------------------------------------------------------------ serving mix
# Viscosity of each job type of the serving mix: the smallest value of the
# ladder {1e-3, 2e-3, 5e-3, 1e-2, 2e-2} (the four-quadrant draws' rule) at
# which the mix's draws of that type run to their last step without an
# equilibrium failure; None keeps the type's own default (the vortex's
# 1e-4 T_inf).
NU_LADDER = (1e-3, 2e-3, 5e-3, 1e-2, 2e-2)
SERVING_NU = {"vortex": None, "quadrant": 1e-3}
# Quadrant draws of the mix whose states, seen in another quadrant's lattice,
# move faster than this are redrawn: the first step rebuilds links at those
# states, and beyond about 1.5 (e.g. |u'| = 1.75 across a diagonal lattice
# jump) the 8-moment D2Q21 equilibrium has no solution, at any viscosity.
SERVING_MAX_LINK_SPEED = 1.5
# Hysteresis half-width of the lattice choice per job type (overlapping
# velocity ranges chosen by history, Sec. III.A.2; 0.5 is the plain
# criterion).  Strong shocks of the quadrant draws otherwise put nodes whose
# lattices differ by two next to each other, and the links rebuilt between
# them leave the equilibrium's envelope at any viscosity of the ladder.
SERVING_HALFWIDTH = {"vortex": 0.5, "quadrant": 0.9}
# Where a state's 8-moment equilibrium has no solution (about 1.8 % of the
# quadrant draws meet one mid-run: rebuilt links whose source moves at |u'|
# 1.3-1.9 in the receiver's lattice, or a node's own state behind a strong
# shock), the serving jobs take the four-constraint equilibrium of that
# state for that solve instead of stopping (lbm_config.fallback).
SERVING_FALLBACK = 1


@dataclasses.dataclass
class JobSpec:
    job_id: int
    kind: str            # "vortex" or "quadrant"
    side: int
    mach: float
    steps: int
    interarrival: float  # unit-rate exponential draw; divide by the rate
    nu: float | None = None   # None: SERVING_NU of the job's type

    def build(self) -> Workload:
        nu = self.nu if self.nu is not None else SERVING_NU[self.kind]
        if self.kind == "vortex":
            wl = isentropic_vortex(self.side, mach=self.mach, steps=self.steps,
                                   seed_index=4, name=f"job{self.job_id}_vortex", nu=nu)
            wl.halfwidth = SERVING_HALFWIDTH["vortex"]
            wl.fallback = SERVING_FALLBACK
            return wl
        wl = four_quadrant(self.side, self.steps, seed_index=4,
                           sub=self.job_id + 1, mach=self.mach, nu=nu,
                           max_link_speed=SERVING_MAX_LINK_SPEED)
        wl.halfwidth = SERVING_HALFWIDTH["quadrant"]
        wl.fallback = SERVING_FALLBACK
        return wl

    @property
    def work(self) -> int:
        return self.side * self.side * self.steps


def serving_jobs(n: int = 10000, seed_index: int = 4) -> List[JobSpec]:
    """Job mix: type vortex/quadrant with p = 1/2, side log-uniform in
    [64, 1024], advection Mach uniform in [0.5, 3], steps uniform in
    {100..2000}, unit-rate exponential inter-arrival gaps."""
    rng = rng_for(seed_index)
    jobs = []
    for j in range(n):
        kind = "vortex" if rng.uniform() < 0.5 else "quadrant"
        side = int(round(math.exp(rng.uniform(math.log(64), math.log(1024)))))
        mach = float(rng.uniform(0.5, 3.0))
        steps = int(rng.integers(100, 2001))
        gap = float(rng.exponential(1.0))
        jobs.append(JobSpec(j, kind, side, mach, steps, gap))
    return jobs


def uniform(nx: int, ny: int, rho: float, ux: float, uy: float, T: float,
            nu: float = 1e-3, steps: int = 10, shift_mode: int = 1,
            fixed_U=(0, 0)) -> Workload:
    f = lambda v: np.full((ny, nx), v, dtype=np.float64)
    return Workload(f"uniform_{nx}x{ny}", nx, ny, f(rho), f(ux), f(uy), f(T), nu,
                    steps, shift_mode, tuple(fixed_U))


def smooth_random(nx: int, ny: int, seed: int, amp=(0.05, 0.2, 0.2, 0.05),
                  base=(1.0, 0.0, 0.0, T0), modes: int = 3, dyadic_bits: int = 0,
                  nu: float = 1e-3, steps: int = 10, shift_mode: int = 0,
                  fixed_U=(0, 0)) -> Workload:
    """Smooth periodic random field: a few low Fourier modes per quantity.

    With dyadic_bits > 0 every value is rounded to a multiple of
    2**-dyadic_bits, so adding or subtracting small integers is exact."""
    rng = np.random.Generator(np.random.PCG64([SEED_BASE, 1000 + seed]))
    x, y = _grid(nx, ny)
    out = []
    for b, a in zip(base, amp):
        acc = np.zeros((ny, nx))
        for _ in range(modes):
            kx = rng.integers(0, 3)
            ky = rng.integers(0, 3) if ny > 1 else 0
            ph = rng.uniform(0, 2 * math.pi)
            acc += np.cos(2 * math.pi * (kx * x / nx + ky * y / ny) + ph)
        v = b + a * acc / modes
        if dyadic_bits:
            v = np.round(v * 2.0 ** dyadic_bits) / 2.0 ** dyadic_bits
        out.append(_c(v))
    return Workload(f"smooth_{nx}x{ny}_{seed}", nx, ny, *out, nu, steps,
                    shift_mode, tuple(fixed_U))


# ------------------------------------------------------------ linear regime
# Sec. IV.B: small perturbations (A = 1e-3) of a uniform flow (rho0 = 1,
# T0 = 0.7), inviscid (nu = 0, so tau = 1/2), periodic.  The mean velocities
# are half-integers or integers; the hysteresis half-width 0.51 (the value
# the paper's runs use) keeps round-off from flipping the lattice of a node
# whose velocity sits on a half-integer.
LINEAR_A = 1e-3
LINEAR_HALFWIDTH = 0.51


def linear_steps(u0: float, L: int = 100, periods: int = 15) -> int:
    """Steps of `periods` flow-through times t_c = L / u0 (Sec. IV.B.1: an
    integer for u0 in {2, 2.5, 3} at L = 100)."""
    t = periods * L / u0
    if abs(t - round(t)) > 1e-9:
        raise ValueError(f"{periods} t_c is not a whole number of steps at u0 = {u0}")
    return int(round(t))


def shear_wave(u0: float, nx: int = 100, steps: int | None = None) -> Workload:
    """Sec. IV.B.1: u_y = A sin(2 pi x / L_x) on a uniform flow u_x = u0,
    nx x 1 nodes; compared after 15 t_c."""
    x, _ = _grid(nx, 1)
    f = lambda v: np.full((1, nx), v, dtype=np.float64)
    steps = linear_steps(u0, nx) if steps is None else steps
    return Workload(f"shear_wave_u{u0:g}", nx, 1, f(RHO0), f(u0),
                    _c(LINEAR_A * np.sin(2 * math.pi * x / nx)), f(T0), 0.0, steps,
                    halfwidth=LINEAR_HALFWIDTH, meta=dict(u0=u0, A=LINEAR_A))


def _spot(L: int):
    x, y = _grid(L, L)
    R = L / 10.0
    return np.exp(-((x - L / 2) ** 2 + (y - L / 2) ** 2) / R ** 2)


def entropy_spot(u0: float, L: int = 100, steps: int | None = None) -> Workload:
    """Sec. IV.B.2: Gaussian hot spot at constant pressure, rho = rho0 (1 -
    A e^{-r^2}), T = T0 (1 + A e^{-r^2}), r^2 = |x - x_c|^2 / R^2, R = L/10,
    centre (L/2, L/2), on u_x = u0; compared after 15 t_c."""
    g = _spot(L)
    f = lambda v: np.full((L, L), v, dtype=np.float64)
    steps = linear_steps(u0, L) if steps is None else steps
    return Workload(f"entropy_spot_u{u0:g}", L, L, _c(RHO0 * (1 - LINEAR_A * g)), f(u0), f(0.0),
                    _c(T0 * (1 + LINEAR_A * g)), 0.0, steps, halfwidth=LINEAR_HALFWIDTH,
                    meta=dict(u0=u0, A=LINEAR_A))


ACOUSTIC_STEPS = 30


def acoustic_pulse(u0: float, L: int = 100, steps: int = ACOUSTIC_STEPS) -> Workload:
    """Sec. IV.B.3: Gaussian pressure pulse P = P0 (1 + A e^{-r^2}) on u_x =
    u0, isentropic: rho = rho0 (P/P0)^{1/gamma}, T = T0 (rho/rho0)^{gamma-1}
    (so that P = rho T); 30 steps.  u0 in {0, 1.3, 2.6, 3.9} (the figure's
    values) moves the pulse by a whole number of nodes in 30 steps."""
    g = _spot(L)
    P0 = RHO0 * T0
    P = P0 * (1 + LINEAR_A * g)
    rho = RHO0 * (P / P0) ** (1.0 / GAMMA)
    T = T0 * (rho / RHO0) ** (GAMMA - 1.0)
    f = lambda v: np.full((L, L), v, dtype=np.float64)
    return Workload(f"acoustic_pulse_u{u0:g}", L, L, _c(rho), f(u0), f(0.0), _c(T), 0.0, steps,
                    halfwidth=LINEAR_HALFWIDTH, meta=dict(u0=u0, A=LINEAR_A))
