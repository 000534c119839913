"""MI355X implementation of the interpolation-free, state-adaptive
compressible lattice Boltzmann step of Coreixas & Latt (arXiv 2009.13426).

Thin Python binding over the C ABI of ``include/lbm.h`` (``liblbm.so``):
PyTorch provides device memory and streams, every step of the method runs
in the library's HIP kernels.  There is no CPU fallback: if the library has
not been built, importing the binding raises.
"""
from __future__ import annotations

import ctypes as C
from typing import Dict, Optional, Sequence

from . import _lib
from ._lib import (ERR_ARG, ERR_HIP, ERR_NEWTON, ERR_NONPHYSICAL, ERR_STATE,  # noqa: F401
                   ERR_WORKSPACE, FP32_STORE, FP64, OK, Q, SHIFT_ADAPTIVE, SHIFT_FIXED,
                   SHIFT_NEIGHBOURHOOD, SHIFT_STATIC)

lib = _lib.load()

PRECISIONS = {"fp64": FP64, "fp32": FP32_STORE, "fp32_store": FP32_STORE,
              FP64: FP64, FP32_STORE: FP32_STORE}
SHIFT_MODES = {"adaptive": SHIFT_ADAPTIVE, "fixed": SHIFT_FIXED, "static": SHIFT_STATIC,
               "neighbourhood": SHIFT_NEIGHBOURHOOD,
               0: SHIFT_ADAPTIVE, 1: SHIFT_FIXED, 2: SHIFT_STATIC, 3: SHIFT_NEIGHBOURHOOD}


class LBMError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = lib.lbm_status_str(status).decode()
        super().__init__(f"{where}: {msg} (status {status})")
        self.status = status


def _check(status: int, where: str):
    if status != OK:
        raise LBMError(status, where)


def velocities(constraints=8):
    """Velocity set in storage order of a constraint count's lattice: D2Q21,
    or D2Q49 for the 13-constraint reference model."""
    cx = (C.c_int32 * 49)()
    cy = (C.c_int32 * 49)()
    q = lib.lbm_lattice_velocities(int(constraints), cx, cy)
    if q == 0:
        raise ValueError(f"no lattice for {constraints} constraints")
    return list(zip(cx[:q], cy[:q]))


def make_config(nx: int, ny: int, precision="fp64", gamma=1.4, nu=0.0, shift_mode="adaptive",
                fixed_U=(0, 0), halfwidth=0.5, newton_tol=1e-12, newton_max_iter=30,
                max_abs_shift=6, sensor=False, stats=False, constraints=8,
                prandtl=1.0, fallback=False) -> _lib.Config:
    cfg = _lib.Config()
    lib.lbm_default_config(C.byref(cfg), int(nx), int(ny))
    cfg.precision = PRECISIONS[precision]
    cfg.gamma = float(gamma)
    cfg.nu = float(nu)
    cfg.shift_mode = SHIFT_MODES[shift_mode]
    cfg.fixed_ux, cfg.fixed_uy = int(fixed_U[0]), int(fixed_U[1])
    cfg.shift_halfwidth = float(halfwidth)
    cfg.newton_tol = float(newton_tol)
    cfg.newton_max_iter = int(newton_max_iter)
    cfg.max_abs_shift = int(max_abs_shift)
    cfg.sensor = int(bool(sensor))
    cfg.collect_stats = int(bool(stats))
    cfg.constraints = int(constraints)
    cfg.prandtl = float(prandtl)
    cfg.fallback = int(bool(fallback))
    return cfg


def workspace_bytes(cfg: _lib.Config) -> int:
    return int(lib.lbm_workspace_bytes(C.byref(cfg)))


class Sim:
    """One periodic nx x ny simulation resident on a GPU."""

    def __init__(self, nx: int, ny: int, device=None, stream=None, like=None, schedule=None,
                 **kw):
        """schedule: None (library default), a dict of lbm_schedule fields,
        or "auto" (the autotuner's cached choice for this size class,
        tuned on a miss; the library default for the four- and
        13-constraint sets, the neighbourhood shift choice and the
        flexible-Prandtl collision, which are built for that schedule
        only)."""
        import torch
        self.torch = torch
        self.device = torch.device("cuda" if device is None else device)
        self.cfg = make_config(nx, ny, **kw)
        self.nx, self.ny = int(nx), int(ny)
        self.Q = 49 if self.cfg.constraints == 13 else Q
        nbytes = workspace_bytes(self.cfg)
        if nbytes == 0:
            raise ValueError(f"invalid configuration {kw} for {nx}x{ny}")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._ctx = C.c_void_p()
        with torch.cuda.device(self.device):
            if like is None:
                st = lib.lbm_create(C.byref(self.cfg), C.c_void_p(self.workspace.data_ptr()),
                                    nbytes, C.c_void_p(self.stream.cuda_stream),
                                    C.byref(self._ctx))
            else:  # initial-guess table copied from another simulation
                st = lib.lbm_create_like(like.handle, C.byref(self.cfg),
                                         C.c_void_p(self.workspace.data_ptr()), nbytes,
                                         C.c_void_p(self.stream.cuda_stream), C.byref(self._ctx))
            _check(st, "lbm_create")
        if schedule == "auto":
            # the four-constraint and neighbourhood-choice kernels are built
            # for the default schedule only
            if int(kw.get("constraints", 8)) != 8 or \
                    float(kw.get("prandtl", 1.0)) not in (0.0, 1.0) or \
                    SHIFT_MODES[kw.get("shift_mode", "adaptive")] == SHIFT_NEIGHBOURHOOD:
                schedule = None
            else:
                from . import autotune
                schedule = autotune.schedule_for(kw.get("precision", "fp64"), nx, ny,
                                                 device=self.device)
        if schedule:
            self.schedule = schedule

    @classmethod
    def from_workload(cls, wl, precision="fp64", device=None, stream=None, like=None,
                      schedule=None, **over):
        kw = dict(nu=wl.nu, gamma=wl.gamma, shift_mode=wl.shift_mode, fixed_U=wl.fixed_U,
                  halfwidth=wl.halfwidth, sensor=wl.sensor, precision=precision,
                  fallback=getattr(wl, "fallback", 0))
        kw.update(over)
        s = cls(wl.nx, wl.ny, device=device, stream=stream, like=like, schedule=schedule, **kw)
        static = wl.static_U if kw["shift_mode"] in (2, "static") else None
        s.init(*wl.fields(), static_U=static)
        return s

    @property
    def handle(self):
        return self._ctx

    def _dev(self, a, dtype):
        t = self.torch.as_tensor(a, dtype=dtype, device=self.device)
        return t.reshape(self.ny, self.nx).contiguous()

    def init(self, rho, ux, uy, T, static_U=None):
        f64 = self.torch.float64
        args = [self._dev(a, f64) for a in (rho, ux, uy, T)]
        ptrs = [C.c_void_p(a.data_ptr()) for a in args]
        with self.torch.cuda.device(self.device):
            if static_U is None:
                st = lib.lbm_init_fields(self._ctx, *ptrs)
            else:
                u8 = [self._dev(a, self.torch.int8) for a in static_U]
                st = lib.lbm_init_fields_static(self._ctx, *ptrs,
                                                *[C.c_void_p(a.data_ptr()) for a in u8])
        _check(st, "lbm_init_fields")
        del args  # lbm_init_fields is synchronous: the fields are consumed

    def step(self, n: int = 1):
        _check(lib.lbm_step(self._ctx, int(n)), "lbm_step")

    def step_async(self, n: int = 1):
        _check(lib.lbm_step_async(self._ctx, int(n)), "lbm_step_async")

    def step_profiled(self, n: int):
        """n steps with HIP events around every launch; returns the summed
        (rebuild, step) launch durations in milliseconds."""
        a, b = C.c_double(), C.c_double()
        _check(lib.lbm_step_profiled(self._ctx, int(n), C.byref(a), C.byref(b)),
               "lbm_step_profiled")
        return a.value, b.value

    def copy_state_from(self, other: "Sim"):
        """Device-to-device copy of `other`'s state into this simulation
        (same configuration required): checkpoint / restore."""
        _check(lib.lbm_copy_state(self._ctx, other.handle), "lbm_copy_state")

    def step_graph(self, n: int, chunk: int = 32):
        """n steps, full chunks as replays of a HIP graph of `chunk` steps
        (lbm_step_graph_async), then waits and checks for errors."""
        _check(lib.lbm_step_graph_async(self._ctx, int(n), int(chunk)), "lbm_step_graph_async")
        self.sync()

    def step_graph_async(self, n: int, chunk: int = 32):
        _check(lib.lbm_step_graph_async(self._ctx, int(n), int(chunk)), "lbm_step_graph_async")

    @property
    def schedule(self) -> Dict[str, int]:
        s = _lib.Schedule()
        _check(lib.lbm_get_schedule(self._ctx, C.byref(s)), "lbm_get_schedule")
        return {k: int(getattr(s, k)) for k, _ in _lib.Schedule._fields_}

    @schedule.setter
    def schedule(self, sched: Dict[str, int]):
        cur = self.schedule
        cur.update({k: int(v) for k, v in sched.items()})
        s = _lib.Schedule(**cur)
        _check(lib.lbm_set_schedule(self._ctx, C.byref(s)), f"lbm_set_schedule {cur}")

    def sync(self):
        _check(lib.lbm_sync(self._ctx), "lbm_sync")

    def macros(self) -> Dict[str, "torch.Tensor"]:
        t = self.torch
        out = {k: t.empty((self.ny, self.nx), dtype=t.float64, device=self.device)
               for k in ("rho", "ux", "uy", "T")}
        out["Ux"] = t.empty((self.ny, self.nx), dtype=t.int8, device=self.device)
        out["Uy"] = t.empty((self.ny, self.nx), dtype=t.int8, device=self.device)
        _check(lib.lbm_get_macros(self._ctx, *[C.c_void_p(out[k].data_ptr()) for k in
                                               ("rho", "ux", "uy", "T", "Ux", "Uy")]),
               "lbm_get_macros")
        return out

    def populations(self):
        t = self.torch
        f = t.empty((self.Q, self.ny, self.nx), dtype=t.float64, device=self.device)
        g = t.empty_like(f)
        _check(lib.lbm_get_populations(self._ctx, C.c_void_p(f.data_ptr()),
                                       C.c_void_p(g.data_ptr())), "lbm_get_populations")
        return f, g

    def diag(self) -> dict:
        d = _lib.Diag()
        _check(lib.lbm_get_diag(self._ctx, C.byref(d)), "lbm_get_diag")
        return dict(steps_done=d.steps_done, status=d.status, fail_step=d.fail_step,
                    fail_node=d.fail_node, newton_calls=d.newton_calls,
                    newton_iters=d.newton_iters, mismatched_links=d.mismatched_links,
                    iter_hist=list(d.iter_hist), conserved=list(d.conserved),
                    fallback_solves=d.fallback_solves)

    def close(self):
        if getattr(self, "_ctx", None) and self._ctx.value:
            lib.lbm_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def step_batched(sims: Sequence[Sim], nsteps: Sequence[int], graph: bool = False):
    """Advances several simulations sharing one stream, nsteps[k] steps each.
    graph: replay the quantum as a HIP graph kept by sims[0]
    (lbm_step_batched_graph); returns 1 if the graph was recorded by this
    call, 0 if it was replayed (None without graph)."""
    n = len(sims)
    arr = (C.c_void_p * n)(*[s.handle.value for s in sims])
    steps = (C.c_int32 * n)(*[int(k) for k in nsteps])
    if not graph:
        _check(lib.lbm_step_batched(arr, steps, n), "lbm_step_batched")
        return None
    built = C.c_int32(0)
    _check(lib.lbm_step_batched_graph(arr, steps, n, C.byref(built)), "lbm_step_batched_graph")
    return built.value


def stream_copy(src, dst, stream=None):
    """Copies the bytes of device tensor src into dst (same byte size) with
    the library's streaming copy kernel, on `stream` (default: torch's
    current stream); asynchronous."""
    import torch
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("stream_copy: src and dst differ in size")
    s = stream if stream is not None else torch.cuda.current_stream(src.device)
    _check(lib.lbm_stream_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()),
                               nbytes, C.c_void_p(s.cuda_stream)), "lbm_stream_copy")
