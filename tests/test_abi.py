"""The C-ABI library loads without a GPU and exports every function that
include/lbm.h declares (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")
LIB = os.path.join(ROOT, "paper_2009_13426_amd", "liblbm.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def so():
    if not os.path.exists(LIB):
        import importlib.util
        spec = importlib.util.spec_from_file_location(
            "_b", os.path.join(ROOT, "paper_2009_13426_amd", "build.py"))
        m = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(m)
        m.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["lbm_create", "lbm_init_fields", "lbm_step", "lbm_get_macros",
                     "lbm_destroy", "lbm_workspace_bytes", "lbm_get_diag",
                     "lbm_step_batched", "lbm_status_str"]:
        assert required in names


def test_every_declared_symbol_is_exported(so):
    missing = [n for n in declared_functions() if not hasattr(so, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_2009_13426_amd import _lib
    assert set(declared_functions()) == set(_lib.SIGNATURES)


def test_host_side_calls_without_gpu(so):
    from paper_2009_13426_amd import _lib
    L = _lib.load()
    cfg = _lib.Config()
    L.lbm_default_config(ctypes.byref(cfg), 64, 32)
    assert cfg.newton_tol == 1e-12 and cfg.gamma == 1.4
    n64 = L.lbm_workspace_bytes(ctypes.byref(cfg))
    cfg.precision = 1
    n32 = L.lbm_workspace_bytes(ctypes.byref(cfg))
    assert n64 > 2 * 2 * 21 * 64 * 32 * 8 and n32 < n64
    cfg.nx = 0
    assert L.lbm_workspace_bytes(ctypes.byref(cfg)) == 0
    cfg.nx = 64
    cfg.shift_halfwidth = 0.4
    assert L.lbm_workspace_bytes(ctypes.byref(cfg)) == 0
    ctx = ctypes.c_void_p()
    cfg.shift_halfwidth = 0.5
    # a null workspace is rejected before any device work
    assert L.lbm_create(ctypes.byref(cfg), None, 0, None, ctypes.byref(ctx)) == _lib.ERR_WORKSPACE
    assert L.lbm_status_str(-5) == b"equilibrium solve did not converge"
    cx = (ctypes.c_int32 * 21)()
    cy = (ctypes.c_int32 * 21)()
    L.lbm_velocities(cx, cy)
    assert sorted(zip(cx, cy)) == sorted(
        [(0, 0)] + [(a * s, b * s) for a, b in [(1, 0), (0, 1), (1, 1), (1, -1), (2, 0), (0, 2),
                                                 (2, 2), (2, -2), (3, 0), (0, 3)] for s in (1, -1)])


def test_size_limits_and_invalid_configs(so):
    """Planes are addressed with 32-bit byte offsets: a configuration whose
    plane would reach 4 GiB is refused (workspace size 0), as are empty grids
    and out-of-range options; the largest accepted planes are just below."""
    from paper_2009_13426_amd import _lib
    L = _lib.load()

    def size(nx, ny, **kw):
        cfg = _lib.Config()
        L.lbm_default_config(ctypes.byref(cfg), nx, ny)
        for k, v in kw.items():
            setattr(cfg, k, v)
        return L.lbm_workspace_bytes(ctypes.byref(cfg))

    assert size(32768, 16384) == 0                      # FP64: 2^29 nodes x 8 B = 4 GiB
    assert size(32768, 16383) > 0
    assert size(32768, 32768, precision=1) == 0         # FP32: 2^30 nodes x 4 B = 4 GiB
    assert size(32768, 32767, precision=1) > 0
    assert size(0, 5) == 0 and size(5, 0) == 0
    assert size(1, 1) > 0
    assert size(8, 8, shift_mode=4) == 0
    assert size(8, 8, shift_mode=3, shift_halfwidth=1.0) == 0
    assert size(8, 8, shift_mode=3, shift_halfwidth=0.9) > 0
    assert size(8, 8, shift_mode=3, shift_halfwidth=0.9, constraints=4) == 0
    assert size(8, 8, constraints=5) == 0 and size(8, 8, constraints=4) > 0
    assert size(8, 8, newton_max_iter=0) == 0
    # the 13-constraint reference model: D2Q49, FP64 only, no neighbourhood choice
    assert size(8, 8, constraints=13) > 2 * 2 * 49 * 64 * 8
    assert size(8, 8, constraints=13, precision=1) == 0
    assert size(8, 8, constraints=13, shift_mode=3, shift_halfwidth=0.9) == 0
    cx = (ctypes.c_int32 * 49)()
    cy = (ctypes.c_int32 * 49)()
    assert L.lbm_lattice_velocities(13, cx, cy) == 49
    assert sorted(zip(cx, cy)) == [(a, b) for a in range(-3, 4) for b in range(-3, 4)]
    assert L.lbm_lattice_velocities(8, cx, cy) == 21 and L.lbm_lattice_velocities(4, None, None) == 21
    assert L.lbm_lattice_velocities(5, cx, cy) == 0
    # the flexible-Prandtl collision: 8 or 13 constraints, no neighbourhood choice
    assert size(8, 8, prandtl=0.71) > 0 and size(8, 8, prandtl=0.0) > 0
    assert size(8, 8, prandtl=-1.0) == 0 and size(8, 8, prandtl=1e-3) == 0
    assert size(8, 8, prandtl=0.71, constraints=4) == 0
    assert size(8, 8, prandtl=0.71, constraints=13) > 0
    assert size(8, 8, prandtl=0.71, constraints=13, precision=1) == 0
    assert size(8, 8, prandtl=0.71, shift_mode=3, shift_halfwidth=0.9) == 0
    assert size(8, 8, max_abs_shift=13) == 0
