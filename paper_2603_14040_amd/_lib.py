"""ctypes view of the C ABI in include/tephra.h (argument marshalling only).

Loading fails loudly if libtephra.so has not been built: there is no CPU or
PyTorch fallback for any entry point.
"""
from __future__ import annotations

import ctypes
import os
import re
from ctypes import POINTER, c_char_p, c_double, c_int32, c_size_t, c_uint64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtephra.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "tephra.h")

TPH_OK, TPH_NOT_CONVERGED = 0, 1
STATUS_NAMES = {0: "TPH_OK", 1: "TPH_NOT_CONVERGED", -1: "TPH_ERR_INVALID", -2: "TPH_ERR_OOM",
                -3: "TPH_ERR_HIP", -4: "TPH_ERR_NONFINITE", -5: "TPH_ERR_UNSUPPORTED"}
FREE_SLIP, NO_SLIP = 0, 1
FP64, MIXED = 0, 1
SMOOTH_JACOBI, SMOOTH_GS, SMOOTH_RAS, SMOOTH_RAS_MIXED = 0, 1, 2, 3
MEAN_ARITHMETIC, MEAN_GEOMETRIC = 0, 1
ACCEL_FGMRES, ACCEL_GCR, ACCEL_ANDERSON = 0, 1, 2
NODES_BASIC, NODES_CELL, NODES_VX, NODES_VY = 0, 1, 2, 3
NODE_KINDS = {"basic": NODES_BASIC, "cell": NODES_CELL, "vx": NODES_VX, "vy": NODES_VY}
ACCEL_NAMES = {"fgmres": ACCEL_FGMRES, "gcr": ACCEL_GCR, "anderson": ACCEL_ANDERSON}
KERNEL_SMOOTH, KERNEL_APPLY, KERNEL_RESIDUAL, KERNEL_RESTRICT, KERNEL_PROLONG = 0, 1, 2, 3, 4
KERNEL_GCR_STEP, KERNEL_AA_MIX, KERNEL_LINK = 5, 6, 7


class Desc(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("lx", c_double), ("ly", c_double),
                ("bc", c_int32 * 4), ("precision", c_int32), ("levels", c_int32),
                ("smoother", c_int32), ("nu_pre", c_int32), ("nu_post", c_int32),
                ("nu_growth", c_double), ("omega", c_double), ("alpha", c_double),
                ("eta_mean", c_int32), ("rtol", c_double), ("restart", c_int32),
                ("max_iters", c_int32), ("uzawa_steps", c_int32), ("fused", c_int32),
                ("msweep", c_int32), ("tile_shape", c_int32), ("coarse_level", c_int32),
                ("accel", c_int32), ("beta", c_double), ("ras_tile", c_int32), ("ras_inner", c_int32),
                ("seed", c_uint64), ("graph", c_int32), ("pad_", c_int32), ("coarsen", c_double)]


class Info(ctypes.Structure):
    _fields_ = [("iters", c_int32), ("restarts", c_int32), ("res_energy", c_double),
                ("res_estimate", c_double), ("t_setup_ms", c_double), ("t_solve_ms", c_double),
                ("history", POINTER(c_double)), ("history_len", c_int32), ("vcycles", c_int32),
                ("res_l2", c_double)]


# device allocator callbacks of tph_set_allocator
ALLOC_FN = ctypes.CFUNCTYPE(c_void_p, c_size_t, c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, c_void_p, c_void_p)


class TephraError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn} failed with {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def header_functions():
    """Names of the functions declared in include/tephra.h."""
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tph_[a-z_0-9]+)\s*\(", src)))


def load(path: str = LIB_PATH):
    """Load libtephra.so and declare every signature; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"HIP library {path} is not built; run `python -m paper_2603_14040_amd.build` "
            "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    P = c_void_p
    sig = {
        "tph_desc_default": (None, [POINTER(Desc), c_int32, c_int32]),
        "tph_create": (c_int32, [POINTER(Desc), P, POINTER(P)]),
        "tph_set_allocator": (c_int32, [P, ALLOC_FN, FREE_FN, P]),
        "tph_set_coefficients": (c_int32, [P, P, P, P, c_double, c_double, P, P]),
        "tph_solve": (c_int32, [P, P, P, P, POINTER(Info)]),
        "tph_solve_rhs": (c_int32, [P, P, P, P, P, P, P, POINTER(Info)]),
        "tph_lithostatic_pressure": (c_int32, [P, P, c_double, P]),
        "tph_solve_continuation": (c_int32, [P, P, P, P, c_double, c_double, POINTER(c_double), c_int32, c_double,
                                             c_int32, P, P, P, POINTER(Info)]),
        "tph_apply": (c_int32, [P, P, P, P, P, P, P]),
        "tph_precondition": (c_int32, [P, P, P, P, P, P, P]),
        "tph_precondition_apply": (c_int32, [P, P, P, P, P, P, P, P, P, P]),
        "tph_energy_residual": (c_int32, [P, P, P, P, POINTER(c_double)]),
        "tph_energy_residual_noalloc": (c_int32, [POINTER(Desc), P, P, P, c_double, c_double, P, P, P, P, P]),
        "tph_level_viscosity": (c_int32, [P, c_int32, P, P]),
        "tph_level_shape": (c_int32, [P, c_int32, POINTER(c_int32), POINTER(c_int32)]),
        "tph_level_plan": (c_int32, [P, c_int32, POINTER(c_int32), POINTER(c_int32)]),
        "tph_solve_adjoint": (c_int32, [P, P, P, P, P, P, P, POINTER(Info)]),
        "tph_coeff_gradient": (c_int32, [P, P, P, P, P, P, P, P, P, P]),
        "tph_time_kernel": (c_int32, [P, c_int32, c_int32, POINTER(c_double), POINTER(c_double)]),
        "tph_kernel_timing": (c_int32, [P, c_int32]),
        "tph_kernel_timing_target": (c_int32, [P, c_int32]),
        "tph_kernel_timing_read": (c_int32, [P, POINTER(c_int32), POINTER(c_double), POINTER(c_double),
                                             POINTER(c_int32)]),
        "tph_destroy": (None, [P]),
        "tph_batch_create": (c_int32, [c_int32, POINTER(Desc), P, POINTER(P)]),
        "tph_batch_set_coefficients": (c_int32, [P, POINTER(P), POINTER(P), POINTER(P), POINTER(c_double)]),
        "tph_batch_solve": (c_int32, [P, POINTER(P), POINTER(P), POINTER(P), POINTER(Info)]),
        "tph_batch_destroy": (None, [P]),
        "tph_markers_create": (c_int32, [c_int32, c_int32, c_double, c_double, c_int32, P, POINTER(P)]),
        "tph_markers_destroy": (None, [P]),
        "tph_markers_bin": (c_int32, [P, c_int32, c_int32, P, P]),
        "tph_markers_to_grid": (c_int32, [P, P, c_double, P]),
        "tph_markers_from_grid": (c_int32, [P, c_int32, c_int32, P, P, P, P]),
        "tph_markers_advect_rk4": (c_int32, [P, c_int32, P, P, P, P, c_double]),
        "tph_markers_sync": (c_int32, [P]),
        "tph_last_error": (c_char_p, []),
        "tph_version": (c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(fn: str, status: int, allow_not_converged: bool = False) -> int:
    if status == TPH_OK or (allow_not_converged and status == TPH_NOT_CONVERGED):
        return status
    msg = _lib.tph_last_error().decode() if _lib is not None else ""
    raise TephraError(fn, status, msg)


def version() -> str:
    return load().tph_version().decode()
