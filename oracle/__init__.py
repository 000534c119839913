"""Python handle on the FP64 CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  It loads ``liblbm_oracle.so`` (built from
``lbm_oracle.c`` by ``oracle/build.py``) through ctypes and adds the parts of
the reference that are plain closed-form mathematics: the exact Riemann
solution of an ideal gas (``oracle.riemann``) and error metrics.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm_oracle.so")

Q = 21
Q49 = 49
M = 8
OK, ERR_ARG, ERR_NEWTON, ERR_NONPHYSICAL = 0, -1, -5, -6
HIST = 128


class Params(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("gamma", C.c_double),
                ("nu", C.c_double), ("shift_mode", C.c_int), ("fixed_ux", C.c_int),
                ("fixed_uy", C.c_int), ("halfwidth", C.c_double),
                ("newton_tol", C.c_double), ("newton_max_iter", C.c_int),
                ("max_abs_shift", C.c_int), ("sensor", C.c_int), ("constraints", C.c_int),
                ("prandtl", C.c_double), ("fallback", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("newton_calls", C.c_long), ("newton_iters", C.c_long),
                ("mismatched_links", C.c_long), ("hist", C.c_long * HIST),
                ("fail_node", C.c_long), ("steps", C.c_long), ("fallbacks", C.c_long)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        L.orc_velocities.argtypes = [ip, ip]
        L.orc_velocities_q.argtypes = [C.c_int, ip, ip]
        L.orc_lattice_of.argtypes = [C.c_int]
        L.orc_lattice_of.restype = C.c_int
        L.orc_equilibrium.argtypes = [C.c_double, C.c_double, C.c_double, dp,
                                      C.c_double, C.c_int, dp, dp, ip]
        L.orc_equilibrium.restype = C.c_int
        L.orc_targets.argtypes = [C.c_double, C.c_double, C.c_double, dp]
        L.orc_equilibrium_m.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, dp,
                                        C.c_double, C.c_int, dp, dp, ip]
        L.orc_equilibrium_m.restype = C.c_int
        L.orc_targets_m.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, dp]
        L.orc_grad_populations.argtypes = [C.POINTER(Params), C.c_double, C.c_double,
                                           C.c_double, C.c_double, dp, dp, C.c_int,
                                           C.c_int, C.c_int, dp, dp]
        L.orc_grad_populations.restype = C.c_int
        L.orc_select.argtypes = [C.c_double, C.c_int, C.c_double]
        L.orc_select.restype = C.c_int
        L.orc_sensor_alpha.argtypes = [C.c_double]
        L.orc_sensor_alpha.restype = C.c_double
        L.orc_create.argtypes = [C.POINTER(Params)]
        L.orc_create.restype = C.c_void_p
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_init.argtypes = [C.c_void_p, dp, dp, dp, dp]
        L.orc_init.restype = C.c_int
        L.orc_set_static_shift.argtypes = [C.c_void_p, ip, ip]
        L.orc_set_static_shift.restype = C.c_int
        L.orc_step.argtypes = [C.c_void_p, C.c_int]
        L.orc_step.restype = C.c_int
        L.orc_macros.argtypes = [C.c_void_p, dp, dp, dp, dp, ip, ip, ip, ip]
        L.orc_populations.argtypes = [C.c_void_p, dp, dp]
        L.orc_conserved.argtypes = [C.c_void_p, dp]
        L.orc_get_stats.argtypes = [C.c_void_p, C.POINTER(Stats)]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def velocities(lattice=Q):
    """Integer velocities of D2Q21 (default) or D2Q49, one row each."""
    cx = np.zeros(lattice, np.int32)
    cy = np.zeros(lattice, np.int32)
    lib().orc_velocities_q(int(lattice), _ip(cx), _ip(cy))
    return np.stack([cx, cy], 1)


def lattice_of(constraints):
    """Lattice a constraint set is solved on: 49 for 13, else 21."""
    return lib().orc_lattice_of(int(constraints))


def targets(ux, uy, T):
    m = np.zeros(M)
    lib().orc_targets(ux, uy, T, _dp(m))
    return m


def equilibrium(ux, uy, T, lam0=None, tol=1e-12, max_iter=100, constraints=M):
    """Weights w (per unit density), multipliers, iterations, status.
    constraints: 8 (eq. 8moments), 4 (mass, momentum, energy) or 13 (the
    reference model on D2Q49; w then holds 49 weights)."""
    w = np.zeros(lattice_of(constraints))
    lam = np.zeros(constraints)
    it = C.c_int(0)
    l0 = None
    if lam0 is not None:
        l0 = np.ascontiguousarray(lam0, dtype=np.float64)
    rc = lib().orc_equilibrium_m(int(constraints), float(ux), float(uy), float(T),
                                 _dp(l0) if l0 is not None else None, tol, max_iter,
                                 _dp(w), _dp(lam), C.byref(it))
    return w, lam, it.value, rc


def targets_m(constraints, ux, uy, T):
    m = np.zeros(constraints)
    lib().orc_targets_m(int(constraints), ux, uy, T, _dp(m))
    return m


def select(u, Uprev, halfwidth=0.5):
    return lib().orc_select(float(u), int(Uprev), float(halfwidth))


def sensor_alpha(eps):
    """Relaxation-time factor alpha(eps) of the kinetic sensor (eq. DeltaAvg)."""
    return lib().orc_sensor_alpha(float(eps))


def make_params(nx, ny, gamma=1.4, nu=1e-3, shift_mode=0, fixed_U=(0, 0),
                halfwidth=0.5, newton_tol=1e-12, newton_max_iter=100,
                max_abs_shift=6, sensor=0, constraints=8, prandtl=1.0, fallback=0) -> Params:
    return Params(nx, ny, gamma, nu, shift_mode, fixed_U[0], fixed_U[1], halfwidth,
                  newton_tol, newton_max_iter, max_abs_shift, sensor, constraints, prandtl,
                  int(fallback))


def grad_populations(params: Params, rho, ux, uy, T, du, dT, L, post):
    q = lattice_of(params.constraints)
    f = np.zeros(q)
    g = np.zeros(q)
    du = np.ascontiguousarray(du, dtype=np.float64)
    dT = np.ascontiguousarray(dT, dtype=np.float64)
    rc = lib().orc_grad_populations(C.byref(params), rho, ux, uy, T, _dp(du), _dp(dT),
                                    int(L[0]), int(L[1]), int(post), _dp(f), _dp(g))
    return f, g, rc


class OracleError(RuntimeError):
    def __init__(self, rc, where):
        super().__init__(f"oracle {where} failed with status {rc}")
        self.rc = rc


class Sim:
    """Periodic nx x ny simulation on the CPU oracle."""

    def __init__(self, nx, ny, **kw):
        self.nx, self.ny = nx, ny
        self.params = make_params(nx, ny, **kw)
        self.Q = lattice_of(self.params.constraints)
        self._h = lib().orc_create(C.byref(self.params))
        if not self._h:
            raise ValueError("invalid oracle parameters")

    @classmethod
    def from_workload(cls, wl, **over):
        kw = dict(gamma=wl.gamma, nu=wl.nu, shift_mode=wl.shift_mode,
                  fixed_U=wl.fixed_U, halfwidth=wl.halfwidth, sensor=wl.sensor,
                  fallback=getattr(wl, "fallback", 0))
        kw.update(over)
        s = cls(wl.nx, wl.ny, **kw)
        if kw["shift_mode"] == 2:
            s.set_static_shift(*wl.static_U)
        s.init(*wl.fields())
        return s

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    def set_static_shift(self, Ux, Uy):
        a = [np.ascontiguousarray(v, dtype=np.int32).reshape(-1) for v in (Ux, Uy)]
        lib().orc_set_static_shift(self._h, *map(_ip, a))

    def init(self, rho, ux, uy, T):
        a = [np.ascontiguousarray(v, dtype=np.float64).reshape(-1) for v in (rho, ux, uy, T)]
        rc = lib().orc_init(self._h, *map(_dp, a))
        if rc:
            raise OracleError(rc, "init")

    def step(self, n=1):
        rc = lib().orc_step(self._h, int(n))
        if rc:
            raise OracleError(rc, "step")

    def macros(self):
        N = self.nx * self.ny
        r, ux, uy, T = (np.zeros(N) for _ in range(4))
        U = [np.zeros(N, np.int32) for _ in range(4)]
        lib().orc_macros(self._h, _dp(r), _dp(ux), _dp(uy), _dp(T), *map(_ip, U))
        sh = (self.ny, self.nx)
        return dict(rho=r.reshape(sh), ux=ux.reshape(sh), uy=uy.reshape(sh),
                    T=T.reshape(sh), Ucx=U[0].reshape(sh), Ucy=U[1].reshape(sh),
                    Unx=U[2].reshape(sh), Uny=U[3].reshape(sh))

    def populations(self):
        N = self.nx * self.ny
        f = np.zeros(self.Q * N)
        g = np.zeros(self.Q * N)
        lib().orc_populations(self._h, _dp(f), _dp(g))
        return f.reshape(self.Q, self.ny, self.nx), g.reshape(self.Q, self.ny, self.nx)

    def conserved(self):
        out = np.zeros(4)
        lib().orc_conserved(self._h, _dp(out))
        return out

    def stats(self):
        st = Stats()
        lib().orc_get_stats(self._h, C.byref(st))
        return dict(newton_calls=st.newton_calls, newton_iters=st.newton_iters,
                    mismatched_links=st.mismatched_links, hist=list(st.hist),
                    fail_node=st.fail_node, steps=st.steps, fallbacks=st.fallbacks)


def rel_err_scalar(a, b):
    """max over nodes of |a - b| / |b| (density, temperature)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b) / np.abs(b)))


def rel_err_vector(ax, ay, bx, by):
    """max |u_a - u_b| / max |u_b| over the field (velocity)."""
    num = np.sqrt((np.asarray(ax) - bx) ** 2 + (np.asarray(ay) - by) ** 2)
    den = np.max(np.sqrt(np.asarray(bx) ** 2 + np.asarray(by) ** 2))
    return float(np.max(num) / den) if den > 0 else float(np.max(num))
