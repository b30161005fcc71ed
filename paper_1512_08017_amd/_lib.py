"""ctypes declarations of the C ABI in include/lsefit.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# LSEFIT_LIB names another build of the same library (the host-sanitized build
# that the CPU sanitizer test loads); by default the in-tree liblsefit.so
LIB_PATH = os.environ.get("LSEFIT_LIB") or os.path.join(HERE, "liblsefit.so")

LSEFIT_MAX_DEGREE = 8
OK, INVALID_ARG, SINGULAR, NONFINITE, WORKSPACE, DEVICE, UNSUPPORTED = range(7)
F32, F64 = 0, 1
PREC_F64, PREC_F32C = 0, 1
SOLVER_GEPP, SOLVER_CHOLESKY = 0, 1
BASIS_MONOMIAL, BASIS_CHEBYSHEV = 0, 1
LSEFIT_MAX_DEGREE_CHEBYSHEV = 16
NOALLOC_SCRATCH_BYTES = 4 << 20   # LSEFIT_NOALLOC_SCRATCH_BYTES
RANGE_GIVEN, RANGE_AUTO = 0, 1
OUTPUT_X, OUTPUT_X_AND_T = 0, 1

STATUS_NAMES = {OK: "ok", INVALID_ARG: "invalid_arg", SINGULAR: "singular", NONFINITE: "nonfinite",
                WORKSPACE: "workspace", DEVICE: "device", UNSUPPORTED: "unsupported"}

# C-ABI symbols the library must export (one per declaration in include/lsefit.h)
EXPORTS = (
    "lsefit_workspace_bytes", "lsefit_default_schedule", "lsefit_set_default_schedule",
    "fit_moments", "fit_solve", "fit_single", "fit_single_noalloc", "fit_qr", "fit_qr_batched", "fit_batched", "fit_backward",
    "fit_residuals",
    "fit_plan_create", "fit_plan_tune", "fit_plan_set_tune_cache", "fit_plan_set_schedule", "fit_plan_get_schedule",
    "fit_plan_set_graph", "fit_plan_get_graph", "fit_plan_destroy", "lsefit_status_string", "lsefit_device_cus",
    "lsefit_timing_enable", "lsefit_timing_reset", "lsefit_timing_read", "lsefit_read_probe", "lsefit_copy_probe",
)


class Options(ctypes.Structure):
    _fields_ = [("degree", ctypes.c_int32), ("precision", ctypes.c_int32), ("refine_steps", ctypes.c_int32),
                ("range_mode", ctypes.c_int32), ("center", ctypes.c_double), ("scale", ctypes.c_double),
                ("solver", ctypes.c_int32), ("basis", ctypes.c_int32), ("output_basis", ctypes.c_int32)]


class Schedule(ctypes.Structure):
    _fields_ = [("waves", ctypes.c_int32), ("waves_per_block", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("unroll", ctypes.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class LsefitError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {STATUS_NAMES.get(code, code)}")


_lib = None
vp = ctypes.c_void_p
i32, i64, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
OptP = ctypes.POINTER(Options)
SchP = ctypes.POINTER(Schedule)


def load():
    """Load liblsefit.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_1512_08017_amd.build; "
                           "the fit has no CPU path")
    L = ctypes.CDLL(LIB_PATH)
    L.lsefit_workspace_bytes.argtypes = [i64, i32, SchP]
    L.lsefit_workspace_bytes.restype = sz
    L.lsefit_default_schedule.argtypes = [SchP]
    L.lsefit_set_default_schedule.argtypes = [SchP]
    L.fit_moments.argtypes = [vp, vp, i64, i32, OptP, vp, sz, vp, vp]
    L.fit_solve.argtypes = [vp, OptP, vp, vp, i64, i32, vp, sz, vp, vp, vp]
    L.fit_single.argtypes = [vp, vp, i64, i32, OptP, vp, sz, vp, vp, vp, vp]
    L.fit_single_noalloc.argtypes = [vp, vp, i64, i32, OptP, vp, vp, vp, vp]
    L.fit_qr.argtypes = [vp, vp, i64, i32, OptP, vp, sz, vp, vp, vp, vp]
    L.fit_qr_batched.argtypes = [vp, vp, vp, vp, i64, i32, OptP, vp, sz, vp, i32, vp, vp, vp]
    L.fit_batched.argtypes = [vp, vp, vp, vp, i64, i32, OptP, vp, vp, sz, vp, i32, vp, vp]
    L.fit_backward.argtypes = [vp, vp, vp, vp, i64, i32, OptP, vp, vp, sz, vp, i32, vp, vp, vp]
    L.fit_residuals.argtypes = [vp, vp, vp, vp, i64, i64, i32, OptP, vp, vp, sz, vp, vp, vp]
    L.fit_plan_create.argtypes = [ctypes.POINTER(vp), i64, i32, i32, i32]
    L.fit_plan_tune.argtypes = [vp, vp, vp, vp, vp, i64, OptP, vp, i32, vp, vp, i32, ctypes.POINTER(ctypes.c_double)]
    L.fit_plan_set_schedule.argtypes = [vp, SchP]
    L.fit_plan_set_tune_cache.argtypes = [vp, ctypes.c_char_p]
    L.fit_plan_get_schedule.argtypes = [vp, SchP]
    L.fit_plan_set_graph.argtypes = [vp, i32]
    L.fit_plan_get_graph.argtypes = [vp, ctypes.POINTER(i32)]
    L.fit_plan_destroy.argtypes = [vp]
    L.fit_plan_destroy.restype = None
    L.lsefit_status_string.argtypes = [i32]
    L.lsefit_status_string.restype = ctypes.c_char_p
    L.lsefit_device_cus.restype = i32
    L.lsefit_timing_enable.argtypes = [i32]
    L.lsefit_read_probe.argtypes = [vp, vp, i64, SchP, i32, i32, vp, sz, vp]
    L.lsefit_copy_probe.argtypes = [vp, vp, vp, vp, i64, SchP, i32, i32, vp]
    L.lsefit_timing_read.argtypes = [i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
    for name in ("lsefit_default_schedule", "lsefit_set_default_schedule", "fit_moments", "fit_solve", "fit_single",
                 "fit_single_noalloc",
                 "fit_qr", "fit_qr_batched", "fit_residuals",
                 "fit_batched", "fit_backward", "fit_plan_create", "fit_plan_tune", "fit_plan_set_tune_cache",
                 "fit_plan_set_schedule",
                 "fit_plan_get_schedule", "fit_plan_set_graph", "fit_plan_get_graph", "lsefit_timing_enable", "lsefit_timing_reset",
                 "lsefit_timing_read", "lsefit_read_probe", "lsefit_copy_probe"):
        getattr(L, name).restype = i32
    _lib = L
    return L


def check(code: int, where: str):
    if code != OK:
        raise LsefitError(code, where)
