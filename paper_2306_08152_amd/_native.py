"""ctypes declarations of the C ABI in include/qfactor.h (argument marshalling
only; every step of the sweep runs in the HIP library)."""
from __future__ import annotations

import ctypes
import os

from .hipbuild import lib_path

QF_OK, QF_EINVAL, QF_EUNSUPPORTED, QF_EHIP, QF_EWORKSPACE, QF_ENUMERIC, QF_ETIMEOUT = 0, -1, -2, -3, -4, -5, -6
QF_C128, QF_C64 = 0, 1
QF_MODE_AUTO, QF_MODE_RESIDENT, QF_MODE_STREAMING = 0, 1, 2
QF_LEFT, QF_RIGHT = 0, 1
QF_CONVERGED, QF_PLATEAU, QF_MAX_ITER, QF_NUMERIC = 0, 1, 2, 3
QF_KIND_U4, QF_KIND_FIXED, QF_KIND_U2, QF_KIND_RZ, QF_KIND_GPI, QF_KIND_MS = 0, 1, 2, 3, 4, 5

EXPORTED = [
    "qf_create", "qf_destroy", "qf_set_stream", "qf_strerror", "qf_last_error", "qf_options_default",
    "qf_workspace_size", "qf_build", "qf_apply_gate", "qf_environment", "qf_optimize_gate",
    "qf_update_gate", "qf_cost", "qf_instantiate", "qf_batch_workspace_size", "qf_instantiate_batch",
    "qf_gradient_workspace_size", "qf_gradient", "qf_su4_gates", "qf_su4_vjp", "qf_lbfgs_options_default",
    "qf_lbfgs_workspace_size", "qf_lbfgs", "qf_set_pass_tile", "qf_delete_gates_workspace_size", "qf_delete_gates",
    "qf_workspace_size3", "qf_instantiate3", "qf_optimize_gate3", "qf_instantiate_noalloc", "qf_set_batch_config", "qf_set_pass2_tiles",
]
QF_NOALLOC_WORKSPACE_BYTES = 64 << 20


class QfOptions(ctypes.Structure):
    _fields_ = [
        ("dist_tol", ctypes.c_double),
        ("diff_tol_a", ctypes.c_double),
        ("diff_tol_r", ctypes.c_double),
        ("long_diff_count", ctypes.c_int32),
        ("long_diff_r", ctypes.c_double),
        ("min_iter", ctypes.c_int32),
        ("max_iter", ctypes.c_int32),
        ("reset_iter", ctypes.c_int32),
        ("beta", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("mode", ctypes.c_int32),
        ("recheck_below", ctypes.c_double),
        ("stream_groups", ctypes.c_int32),
        ("gate_kinds", ctypes.POINTER(ctypes.c_int32)),
        ("gate_pairs", ctypes.c_int32),
    ]


class QfStats(ctypes.Structure):
    _fields_ = [
        ("sweeps", ctypes.c_int32),
        ("best_start", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("n_resets", ctypes.c_int32),
        ("n_rechecks", ctypes.c_int32),
        ("mode_used", ctypes.c_int32),
        ("best_cost", ctypes.c_double),
        ("elapsed_ms", ctypes.c_double),
        ("cost_history", ctypes.POINTER(ctypes.c_double)),
        ("cost_history_rows", ctypes.c_int32),
        ("timing", ctypes.c_int32),
        ("pass_launches", ctypes.c_int32),
        ("env_launches", ctypes.c_int32),
        ("pass_ms", ctypes.c_double),
        ("env_ms", ctypes.c_double),
        ("sweep_ms", ctypes.c_double),
        ("pass_tcols", ctypes.c_int32),
        ("pass2_launches", ctypes.c_int32),
        ("pass2_ms", ctypes.c_double),
        ("batch_slots", ctypes.c_int32),
        ("batch_wg_per_cu", ctypes.c_int32),
    ]


class QfLbfgsResult(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int32),
        ("evaluations", ctypes.c_int32),
        ("best_start", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("best_cost", ctypes.c_double),
        ("elapsed_ms", ctypes.c_double),
        ("cost_history", ctypes.POINTER(ctypes.c_double)),
        ("cost_history_rows", ctypes.c_int32),
    ]


class QfDeleteResult(ctypes.Structure):
    _fields_ = [
        ("attempts", ctypes.c_int32),
        ("deleted", ctypes.c_int32),
        ("sweeps", ctypes.c_int32),
        ("elapsed_ms", ctypes.c_double),
    ]


class QfLbfgsOptions(ctypes.Structure):
    _fields_ = [
        ("history", ctypes.c_int32),
        ("max_iter", ctypes.c_int32),
        ("max_ls", ctypes.c_int32),
        ("c1", ctypes.c_double),
        ("grad_tol", ctypes.c_double),
        ("ftol_r", ctypes.c_double),
        ("precision", ctypes.c_int32),
    ]


_VP = ctypes.c_void_p
_I32P = ctypes.POINTER(ctypes.c_int32)
_DP = ctypes.POINTER(ctypes.c_double)

_SIGS = {
    "qf_create": (ctypes.c_int, [ctypes.POINTER(_VP), ctypes.c_int, _VP]),
    "qf_destroy": (ctypes.c_int, [_VP]),
    "qf_set_stream": (ctypes.c_int, [_VP, _VP]),
    "qf_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "qf_last_error": (ctypes.c_char_p, [_VP]),
    "qf_options_default": (None, [ctypes.POINTER(QfOptions)]),
    "qf_workspace_size": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(QfOptions)]),
    "qf_build": (ctypes.c_int, [_VP, ctypes.c_int, _VP, ctypes.c_int, _I32P, _VP, ctypes.c_int, ctypes.c_int, _VP]),
    "qf_apply_gate": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, _VP, ctypes.c_int, _I32P, _VP, ctypes.c_int,
                                     ctypes.c_int]),
    "qf_environment": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, _VP, ctypes.c_int, _I32P, _VP]),
    "qf_optimize_gate": (ctypes.c_int, [_VP, ctypes.c_int, _VP, _VP, ctypes.c_double, _VP]),
    "qf_update_gate": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, _VP, ctypes.c_int, _I32P, ctypes.c_int,
                                      ctypes.c_double, _VP, _VP]),
    "qf_cost": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, _VP, ctypes.c_int, _DP, _VP]),
    "qf_instantiate": (ctypes.c_int, [_VP, ctypes.c_int, _VP, ctypes.c_int, _I32P, _VP, ctypes.c_int,
                                      ctypes.c_double, ctypes.POINTER(QfOptions), _VP, ctypes.c_size_t, _VP, _VP,
                                      _DP, ctypes.POINTER(QfStats)]),
    "qf_instantiate_noalloc": (ctypes.c_int, [_VP, ctypes.c_int, _VP, ctypes.c_int, _I32P, _VP, ctypes.c_int,
                                              ctypes.c_double, ctypes.POINTER(QfOptions), _VP, _VP, _DP,
                                              ctypes.POINTER(QfStats)]),
    "qf_workspace_size3": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(QfOptions)]),
    "qf_instantiate3": (ctypes.c_int, [_VP, ctypes.c_int, _VP, ctypes.c_int, _I32P, _VP, ctypes.c_int,
                                       ctypes.c_double, ctypes.POINTER(QfOptions), _VP, ctypes.c_size_t, _VP, _VP,
                                       _DP, ctypes.POINTER(QfStats)]),
    "qf_optimize_gate3": (ctypes.c_int, [_VP, ctypes.c_int, _VP, _VP, ctypes.c_double, _VP]),
    "qf_batch_workspace_size": (ctypes.c_size_t, [ctypes.c_int, _I32P, _I32P, ctypes.c_int,
                                                  ctypes.POINTER(QfOptions)]),
    "qf_instantiate_batch": (ctypes.c_int, [_VP, ctypes.c_int, _I32P, _I32P, _I32P, _VP, _VP, ctypes.c_int,
                                            ctypes.c_double, ctypes.POINTER(QfOptions), _VP, ctypes.c_size_t, _VP,
                                            _DP, _I32P, _I32P, _I32P, ctypes.POINTER(QfStats)]),
    "qf_gradient_workspace_size": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "qf_gradient": (ctypes.c_int, [_VP, ctypes.c_int, _VP, ctypes.c_int, _I32P, _VP, ctypes.c_int, ctypes.c_int,
                                   _VP, ctypes.c_size_t, _VP, _VP]),
    "qf_su4_gates": (ctypes.c_int, [_VP, ctypes.c_int, _VP, _VP]),
    "qf_su4_vjp": (ctypes.c_int, [_VP, ctypes.c_int, _VP, _VP, _VP]),
    "qf_lbfgs_options_default": (None, [ctypes.POINTER(QfLbfgsOptions)]),
    "qf_set_pass_tile": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "qf_set_batch_config": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "qf_set_pass2_tiles": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "qf_delete_gates_workspace_size": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                         ctypes.POINTER(QfOptions)]),
    "qf_delete_gates": (ctypes.c_int, [_VP, ctypes.c_int, _VP, ctypes.c_int, _I32P, _VP, _VP, ctypes.c_int,
                                       ctypes.c_double, ctypes.POINTER(QfOptions), _VP, ctypes.c_size_t, _I32P, _VP,
                                       _DP, ctypes.POINTER(QfDeleteResult)]),
    "qf_lbfgs_workspace_size": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                  ctypes.POINTER(QfLbfgsOptions)]),
    "qf_lbfgs": (ctypes.c_int, [_VP, ctypes.c_int, _VP, ctypes.c_int, _I32P, _VP, ctypes.c_int, ctypes.c_double,
                                ctypes.POINTER(QfLbfgsOptions), _VP, ctypes.c_size_t, _VP, _DP,
                                ctypes.POINTER(QfLbfgsResult)]),
}

_lib = None


def load(path: str | None = None):
    """Load the built library (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or lib_path()
    if not os.path.exists(p):
        raise RuntimeError(f"HIP library not built: {p} is missing (run paper_2306_08152_amd.hipbuild.build())")
    lib = ctypes.CDLL(p)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib


class QfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (status {code})")
        self.code = code


def check(code: int, ctx=None):
    if code != QF_OK:
        lib = load()
        detail = lib.qf_last_error(ctx).decode() if ctx else ""
        raise QfError(code, f"{lib.qf_strerror(code).decode()}: {detail}")
