"""ctypes declarations of the C ABI in include/lbm.h (argument marshalling only)."""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

Q = 21
HIST_BINS = 32

OK, ERR_ARG, ERR_WORKSPACE, ERR_HIP, ERR_STATE, ERR_NEWTON, ERR_NONPHYSICAL = 0, -1, -2, -3, -4, -5, -6
FP64, FP32_STORE = 0, 1
SHIFT_ADAPTIVE, SHIFT_FIXED, SHIFT_STATIC, SHIFT_NEIGHBOURHOOD = 0, 1, 2, 3


class Config(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("precision", C.c_int32),
                ("gamma", C.c_double), ("nu", C.c_double), ("shift_mode", C.c_int32),
                ("fixed_ux", C.c_int32), ("fixed_uy", C.c_int32),
                ("shift_halfwidth", C.c_double), ("newton_tol", C.c_double),
                ("newton_max_iter", C.c_int32), ("max_abs_shift", C.c_int32),
                ("sensor", C.c_int32), ("collect_stats", C.c_int32), ("constraints", C.c_int32),
                ("prandtl", C.c_double), ("fallback", C.c_int32)]


class Diag(C.Structure):
    _fields_ = [("steps_done", C.c_int64), ("status", C.c_int32), ("fail_step", C.c_int32),
                ("fail_node", C.c_int64), ("newton_calls", C.c_int64),
                ("newton_iters", C.c_int64), ("mismatched_links", C.c_int64),
                ("iter_hist", C.c_int64 * HIST_BINS), ("conserved", C.c_double * 4),
                ("fallback_solves", C.c_int64)]


class Schedule(C.Structure):
    _fields_ = [("step_block", C.c_int32), ("tiles_per_block", C.c_int32),
                ("xcd_remap", C.c_int32), ("rebuild_blocks", C.c_int32)]


# name -> (restype, argtypes); every function the header declares
SIGNATURES = {
    "lbm_default_config": (None, [C.POINTER(Config), C.c_int32, C.c_int32]),
    "lbm_workspace_bytes": (C.c_size_t, [C.POINTER(Config)]),
    "lbm_create": (C.c_int, [C.POINTER(Config), C.c_void_p, C.c_size_t, C.c_void_p,
                             C.POINTER(C.c_void_p)]),
    "lbm_create_like": (C.c_int, [C.c_void_p, C.POINTER(Config), C.c_void_p, C.c_size_t,
                                  C.c_void_p, C.POINTER(C.c_void_p)]),
    "lbm_init_fields": (C.c_int, [C.c_void_p] + [C.c_void_p] * 4),
    "lbm_init_fields_static": (C.c_int, [C.c_void_p] + [C.c_void_p] * 6),
    "lbm_step": (C.c_int, [C.c_void_p, C.c_int32]),
    "lbm_step_async": (C.c_int, [C.c_void_p, C.c_int32]),
    "lbm_step_profiled": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_double),
                                    C.POINTER(C.c_double)]),
    "lbm_copy_state": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lbm_set_schedule": (C.c_int, [C.c_void_p, C.POINTER(Schedule)]),
    "lbm_get_schedule": (C.c_int, [C.c_void_p, C.POINTER(Schedule)]),
    "lbm_step_graph_async": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    "lbm_sync": (C.c_int, [C.c_void_p]),
    "lbm_get_macros": (C.c_int, [C.c_void_p] + [C.c_void_p] * 6),
    "lbm_get_populations": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "lbm_velocities": (None, [C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "lbm_lattice_velocities": (C.c_int32, [C.c_int32, C.POINTER(C.c_int32),
                                           C.POINTER(C.c_int32)]),
    "lbm_get_diag": (C.c_int, [C.c_void_p, C.POINTER(Diag)]),
    "lbm_step_batched": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(C.c_int32), C.c_int32]),
    "lbm_step_batched_noalloc": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(C.c_int32),
                                           C.c_int32]),
    "lbm_step_batched_graph": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(C.c_int32),
                                         C.c_int32, C.POINTER(C.c_int32)]),
    "lbm_stream_copy": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "lbm_destroy": (None, [C.c_void_p]),
    "lbm_status_str": (C.c_char_p, [C.c_int]),
}

_lib = None


class LibraryMissing(ImportError):
    pass


def load():
    """Loads liblbm.so; raises LibraryMissing if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LibraryMissing(
                f"{LIB_PATH} not found: build it with `python paper_2009_13426_amd/build.py` "
                "(or __graft_entry__.build()); there is no fallback implementation")
        # PyTorch ships its own HIP runtime.  It must be loaded before this
        # library, so that the library binds to it: a second runtime in the
        # process would not know the device memory torch allocates.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib
