"""ctypes view of librve (include/rve.h). Loading fails loudly when the
library has not been built: there is no fallback path."""
from __future__ import annotations

import ctypes
import os

# RVE_LIBRARY may name another build of the same library (the host-sanitizer
# build, librve_asan.so, for the argument-check tests)
LIB_PATH = os.environ.get("RVE_LIBRARY") or os.path.join(os.path.dirname(os.path.abspath(__file__)), "librve.so")

# Iterations per update of the PCG iterate from the ring of search directions
# (RVE_DIRECTION_RING in the header).
DIRECTION_RING = 8

# enum rve_status
OK, NOT_CONVERGED, BREAKDOWN, EINVAL, EHIP, ENOMEM = 0, 1, 2, -1, -2, -3
# enum rve_precision
FP64, MIX_FP32, MIX_BF16, MIX_FP16 = 0, 1, 2, 3
STENCIL_FP64, STENCIL_FP32 = 0, 1
# enum rve_scheme
SCHEME_Q1, SCHEME_FD5 = 0, 1

EXPORTS = (
    "rve_default_opts", "rve_create", "rve_destroy", "rve_set_stream",
    "rve_solve_batch", "rve_solve_uneven", "rve_grad", "rve_stats",
    "rve_status_string", "rve_set_timing", "rve_last_timing",
    "rve_apply_operator", "rve_apply_precond", "rve_set_autotune", "rve_get_tuned",
    "rve_set_graphs", "rve_force_variants", "rve_sample_lattice", "rve_dos_moments", "rve_dos_eval",
    "rve_solve_batch_3d", "rve_apply_operator_3d", "rve_apply_precond_3d", "rve_set_small_solver",
    "rve_solve", "rve_field_from_mask", "rve_dos_plan", "rve_dos_probes", "rve_occupancy_threshold",
    "rve_grad_noalloc", "rve_sample_fixed_count", "rve_set_direction_update", "rve_set_direction_bf16",
)


class RveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxit", ctypes.c_int), ("prec", ctypes.c_int),
                ("flexible", ctypes.c_int), ("check_every", ctypes.c_int), ("stencil_prec", ctypes.c_int),
                ("scheme", ctypes.c_int)]


_lib = None

_vp = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double


def _declare(lib):
    lib.rve_default_opts.argtypes = [ctypes.POINTER(RveOpts)]
    lib.rve_default_opts.restype = None
    lib.rve_create.argtypes = [ctypes.POINTER(_vp), _i, _vp]
    lib.rve_destroy.argtypes = [_vp]
    lib.rve_set_stream.argtypes = [_vp, _vp]
    lib.rve_solve_batch.argtypes = [_vp, _i, _i, _d, _vp, ctypes.POINTER(RveOpts),
                                    _vp, _vp, _vp, _vp, _vp, _vp]
    lib.rve_solve_batch_3d.argtypes = [_vp, _i, _i, _d, _vp, ctypes.POINTER(RveOpts),
                                       _vp, _vp, _vp, _vp, _vp, _vp]
    lib.rve_apply_operator_3d.argtypes = [_vp, _i, _i, _vp, _vp, _vp]
    lib.rve_apply_precond_3d.argtypes = [_vp, _i, _i, _vp, _vp, _vp, _i]
    lib.rve_solve_uneven.argtypes = [_vp, _i, ctypes.POINTER(_i), ctypes.POINTER(ctypes.c_int64),
                                     _d, _vp, ctypes.POINTER(RveOpts), _vp, _vp, _vp, _vp, _vp, _vp]
    lib.rve_solve.argtypes = [_vp, _i, _d, _vp, ctypes.POINTER(RveOpts), _vp, ctypes.POINTER(_d),
                              ctypes.POINTER(_d), ctypes.POINTER(_i), ctypes.POINTER(_d)]
    lib.rve_grad.argtypes = [_vp, _i, _i, _vp, _vp, _d, _vp, _vp, _vp, _d, _vp, _vp, _i]
    lib.rve_grad_noalloc.argtypes = [_vp, _i, _i, _vp, _vp, _d, _vp, _vp, _vp, _d, _vp, _vp, _i]
    lib.rve_field_from_mask.argtypes = [_vp, _i, ctypes.c_longlong, _vp, _vp, _d, _vp]
    lib.rve_dos_plan.argtypes = [_vp, _i, _i, _i, _vp, _d, ctypes.POINTER(_d), ctypes.POINTER(_i)]
    lib.rve_dos_probes.argtypes = [_vp, _i, _i, _i, ctypes.c_uint64, _vp]
    lib.rve_occupancy_threshold.argtypes = [_d]
    lib.rve_sample_fixed_count.argtypes = [_vp, _i, _i, _i, ctypes.c_uint64, ctypes.c_int64, _i, _d, _d, _vp]
    lib.rve_stats.argtypes = [_vp, _i, _d, _vp, _vp]
    lib.rve_status_string.argtypes = [_i]
    lib.rve_status_string.restype = ctypes.c_char_p
    lib.rve_set_timing.argtypes = [_vp, _i]
    lib.rve_last_timing.argtypes = [_vp, ctypes.POINTER(_d), ctypes.POINTER(ctypes.c_longlong)]
    lib.rve_apply_operator.argtypes = [_vp, _i, _i, _vp, _vp, _vp, _i]
    lib.rve_apply_precond.argtypes = [_vp, _i, _i, _vp, _vp, _vp, _i, _i]
    lib.rve_set_autotune.argtypes = [_vp, _i]
    lib.rve_get_tuned.argtypes = [_vp, _i, _i, _i, _i, ctypes.POINTER(_i)]
    lib.rve_set_graphs.argtypes = [_vp, _i]
    lib.rve_set_small_solver.argtypes = [_vp, _i]
    lib.rve_set_direction_update.argtypes = [_vp, _i]
    lib.rve_set_direction_bf16.argtypes = [_vp, _i]
    lib.rve_force_variants.argtypes = [_vp, _i, _i, _i]
    lib.rve_dos_moments.argtypes = [_vp, _i, _i, _i, _vp, _i, _vp, _d, _i, _vp]
    lib.rve_dos_eval.argtypes = [_vp, _i, _i, _i, _vp, _d, _d, _i, _i, _vp, _vp]
    lib.rve_sample_lattice.argtypes = [_vp, _i, _i, _i, ctypes.c_uint64, ctypes.c_int64, ctypes.c_uint32,
                                       _d, _d, _vp]
    for name in EXPORTS:
        if name not in ("rve_default_opts", "rve_status_string", "rve_occupancy_threshold"):
            getattr(lib, name).restype = _i
    lib.rve_occupancy_threshold.restype = ctypes.c_uint32
    return lib


def lib():
    """The loaded librve; raises if the shared library is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"librve not built ({LIB_PATH} missing): run __graft_entry__.build() "
                "or python -m paper_1903_12227_amd.build")
        _lib = _declare(ctypes.CDLL(LIB_PATH))
    return _lib


def status_string(code: int) -> str:
    return lib().rve_status_string(int(code)).decode()


class RveError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {status_string(code)} ({code})")
        self.code = code


def check(code: int, what: str) -> int:
    """Raise on errors (negative codes); return warnings (>= 0) unchanged."""
    if code < 0:
        raise RveError(code, what)
    return code
