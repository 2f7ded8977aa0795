"""ctypes declarations of the C ABI in include/sbp.h (argument marshalling only)."""

from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# SBP_LIBRARY_VARIANT=poison or asan loads a debug build of the same sources (see build.py)
_VARIANT = os.environ.get("SBP_LIBRARY_VARIANT", "")
if _VARIANT not in ("", "default", "poison", "asan"):
    raise RuntimeError(f"SBP_LIBRARY_VARIANT={_VARIANT!r}: expected poison or asan")
LIB_PATH = os.path.join(_HERE, "libsbp.so" if _VARIANT in ("", "default") else f"libsbp_{_VARIANT}.so")

SBP_OK = 0
STATUS_NAMES = {0: "SBP_OK", 1: "SBP_E_ARG", 2: "SBP_E_SIZE", 3: "SBP_E_NOMEM", 4: "SBP_E_WORKSPACE",
                5: "SBP_E_HIP", 6: "SBP_E_STATE"}
SBP_FP64, SBP_FP32 = 0, 1
SBP_VGF, SBP_SASHA = 0, 1
SBP_REMAP_SPECTRAL, SBP_REMAP_LINEAR = 0, 1
SBP_FLAG_GRAPH, SBP_FLAG_AUTOTUNE, SBP_FLAG_PLAIN, SBP_FLAG_FIVE_PASS, SBP_FLAG_FUSED = 0x1, 0x2, 0x4, 0x8, 0x10

# every symbol include/sbp.h declares
EXPORTS = ("sbp_plan_create", "sbp_workspace_size", "sbp_set_workspace", "sbp_solve", "sbp_plan_destroy",
           "sbp_status_str", "sbp_last_error", "sbp_profile_enable", "sbp_profile_read", "sbp_plan_describe",
           "sbp_ghosts", "sbp_gravity", "sbp_solve_static")
SBP_STATIC_WORKSPACE_BYTES = 128 << 20


class SbpBox(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("lz", ctypes.c_double),
                ("pad", ctypes.c_int32), ("alpha", ctypes.c_double), ("method", ctypes.c_int32),
                ("remap", ctypes.c_int32)]


class SbpShear(ctypes.Structure):
    _fields_ = [("q", ctypes.c_double), ("omega", ctypes.c_double), ("t", ctypes.c_double), ("G", ctypes.c_double)]


_lib = None


def load() -> ctypes.CDLL:
    """Load libsbp.so (built in-tree).  Raises if it is missing: there is no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32, u32 = ctypes.c_int32, ctypes.c_uint32
    lib.sbp_plan_create.argtypes = [ctypes.POINTER(SbpBox), i32, i32, i32, u32, ctypes.POINTER(P)]
    lib.sbp_plan_create.restype = ctypes.c_int
    lib.sbp_workspace_size.argtypes = [P, ctypes.POINTER(ctypes.c_size_t)]
    lib.sbp_workspace_size.restype = ctypes.c_int
    lib.sbp_set_workspace.argtypes = [P, P, ctypes.c_size_t]
    lib.sbp_set_workspace.restype = ctypes.c_int
    lib.sbp_solve.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(SbpShear), P]
    lib.sbp_solve.restype = ctypes.c_int
    lib.sbp_solve_static.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(SbpShear), P]
    lib.sbp_solve_static.restype = ctypes.c_int
    lib.sbp_plan_destroy.argtypes = [P]
    lib.sbp_plan_destroy.restype = ctypes.c_int
    lib.sbp_status_str.argtypes = [ctypes.c_int]
    lib.sbp_status_str.restype = ctypes.c_char_p
    lib.sbp_last_error.argtypes = []
    lib.sbp_last_error.restype = ctypes.c_char_p
    lib.sbp_profile_enable.argtypes = [P, i32]
    lib.sbp_profile_enable.restype = ctypes.c_int
    lib.sbp_profile_read.argtypes = [P, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(ctypes.c_double), i32, ctypes.POINTER(i32)]
    lib.sbp_profile_read.restype = ctypes.c_int
    lib.sbp_plan_describe.argtypes = [P, ctypes.c_char_p, ctypes.c_size_t]
    lib.sbp_plan_describe.restype = ctypes.c_int
    lib.sbp_ghosts.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(P), i32, P]
    lib.sbp_ghosts.restype = ctypes.c_int
    lib.sbp_gravity.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P),
                                ctypes.POINTER(SbpShear), P]
    lib.sbp_gravity.restype = ctypes.c_int
    _lib = lib
    return lib
