"""ctypes loader for ``libwn.so`` (the C ABI in ``include/wn.h``).

The library is looked up next to this file (built in-tree by
``paper_2408_04466_amd.build``).  There is no fallback: if the library is
missing or fails to load, every entry point raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("WN_LIBRARY", os.path.join(HERE, "libwn.so"))

WN_OK = 0
WN_CHI_INVALID = -(2 ** 31)
WN_MAX_LOOPS = 256

_lib = None


class WnError(RuntimeError):
    def __init__(self, status: int, func: str, msg: str):
        super().__init__(f"{func} failed: {msg} (status {status})")
        self.status = status


P = C.c_void_p
I32 = C.c_int32
I64 = C.c_int64
PD = C.POINTER(C.c_double)
PI64 = C.POINTER(C.c_int64)

SIGNATURES = {
    "wn_version": (I32, []),
    "wn_status_string": (C.c_char_p, [I32]),
    "wn_last_error": (C.c_char_p, []),
    "wn_boundary_loops": (I32, [P, I64, I64, P, P, I64, PI64, C.POINTER(I32)]),
    "wn_build_bvh": (I32, [P, I64, P, I64, PD, P, C.POINTER(P)]),
    "wn_free_bvh": (I32, [P]),
    "wn_bvh_direction": (I32, [P, PD]),
    "wn_eval_3d": (I32, [P, P, PI64, I32, P, P, P, I64, P, P, P]),
    "wn_eval_3d_boundary": (I32, [P, P, PI64, I32, P, P, P, I64, P, P, P]),
    "wn_eval_3d_grid": (I32, [P, P, PI64, I32, P, P, P, I64, I64, I64, P, P, P]),
    "wn_eval_3d_curves": (I32, [P, P, I64, P, P, P, I64, P, P, P, P]),
    "wn_eval_3d_patches": (I32, [PD, P, I64, P, I64, P, P, P, I64, P, P, P]),
    "wn_backward_curves": (I32, [P, I64, P, P, P, I64, P, P, P, P]),
    "wn_spatial_order": (I32, [P, P, P, I64, P, P]),
    "wn_diagnose": (I32, [P, P, P, P, I64, P, P]),
    "wn_device_info": (I32, [P, P]),
    "wn_patch_batch_create": (I32, [P, I32, P, P]),
    "wn_patch_batch_free": (I32, [P]),
    "wn_eval_3d_patches_batched": (I32, [P, P, P, P, P, P, P, P, P]),
    "wn_crossings_3d": (I32, [P, P, P, P, I64, P, P]),
    "wn_backward": (I32, [P, PI64, I32, P, P, P, I64, P, P, P, P]),
    "wn_backward_noalloc": (I32, [P, PI64, I32, P, P, P, I64, P, P, P, P]),
    "wn_eval_2d": (I32, [I32, P, I64, PI64, P, I32, I32, P, P, I64, I64, P, P, P]),
    "wn_backward_2d": (I32, [I32, P, I64, PI64, P, I32, I32, P, P, I64, I64, P, P, P, P]),
    "wn_batch2d_create": (I32, [I32, P, I32, P, C.POINTER(P)]),
    "wn_batch2d_free": (I32, [P]),
    "wn_eval_2d_batched": (I32, [P, P, P, P, P, P, P]),
    "wn_batch_create": (I32, [P, I32, PD, I32, P, C.POINTER(P)]),
    "wn_batch_free": (I32, [P]),
    "wn_eval_batched": (I32, [P, P, P, P, P, P, P]),
    "wn_backward_batched": (I32, [P, P, P, P, P, P, P, P]),
    "wn_batch_info": (I32, [P, PI64]),
}


class Surface(C.Structure):
    """Mirror of ``wn_surface`` in include/wn.h."""
    _fields_ = [("V", P), ("nv", I64), ("F", P), ("nf", I64), ("bnd_xyz", P),
                ("loop_off", PI64), ("nloops", I32), ("nq", I64)]


class CurveSet2D(C.Structure):
    """Mirror of ``wn_curveset_2d`` in include/wn.h."""
    _fields_ = [("nseg", I64), ("loop_off", PI64), ("loop_closed", P), ("nloops", I32),
                ("nx", I64), ("ny", I64)]


class PatchSurface(C.Structure):
    """Mirror of ``wn_patch_surface`` in include/wn.h."""
    _fields_ = [("npatch", I64), ("ncurves", I64), ("nq", I64), ("dir", C.c_double * 3)]


def lib():
    """The loaded library (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"libwn.so not found at {LIB_PATH}; build it with "
                "`python -m paper_2408_04466_amd.build` (there is no fallback path)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(status: int, func: str):
    if status != WN_OK:
        msg = lib().wn_last_error().decode(errors="replace")
        raise WnError(status, func, msg)


def exported_symbols():
    return list(SIGNATURES)
