"""MI355X-native QFactor instantiation sweep (arXiv 2306.08152).

The computation lives in the HIP library libqfactor_mi355x.so behind the C ABI
of include/qfactor.h; this package only marshals torch tensors to it.  There is
no CPU fallback: the calls raise if the library is not built or no GPU is
present.
"""
import importlib

from ._native import (  # noqa: F401
    QF_C128, QF_C64, QF_MODE_AUTO, QF_MODE_RESIDENT, QF_MODE_STREAMING, QF_LEFT, QF_RIGHT,
    QF_CONVERGED, QF_PLATEAU, QF_MAX_ITER, QF_NUMERIC, QfError, QfOptions, QfStats, QfLbfgsOptions, load,
)
from .hipbuild import build as build_library, lib_path  # noqa: F401

_API = ("build", "apply_gate", "environment", "optimize_gate", "update_gate", "cost", "instantiate",
        "default_options", "workspace_size", "Result", "instantiate_batch", "pack_batch",
        "batch_workspace_size", "BatchResult", "gradient", "cost_fn", "su4_gates", "su4_vjp", "su4",
        "lbfgs", "lbfgs_options", "LbfgsResult", "set_pass_tile", "set_pass2_tiles", "set_batch_config", "delete_gates", "DeletionResult",
        "instantiate3", "optimize_gate3", "cost_of_gates")


def __getattr__(name):
    # torch-facing wrappers are imported on first use so that importing the
    # package stays cheap on machines without a GPU.
    if name in _API:
        return getattr(importlib.import_module(__name__ + ".api"), name)
    raise AttributeError(name)
