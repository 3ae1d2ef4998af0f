"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/qfactor.h declares, and its host-only logic
(defaults, workspace sizing, argument validation) behaves as documented."""
import ctypes
import json
import os
import re

import pytest

import paper_2306_08152_amd as pkg
from paper_2306_08152_amd import _native as nat

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qfactor.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(pkg.lib_path()):
        pkg.build_library()
    return nat.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qf_[a-z0-9_]+)\s*\(", text)))


def test_header_declarations_match_binding_list():
    assert declared_functions() == sorted(nat.EXPORTED)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_options_default_match_paper(lib):
    with open(os.path.join(ROOT, "tests", "golden", "default_hyperparameters.json")) as f:
        ref = json.load(f)
    o = nat.QfOptions()
    lib.qf_options_default(ctypes.byref(o))
    for k in ("dist_tol", "diff_tol_a", "diff_tol_r", "long_diff_count", "long_diff_r", "min_iter",
              "max_iter", "reset_iter", "beta"):
        assert getattr(o, k) == ref[k], k
    assert o.precision == nat.QF_C128 and o.mode == nat.QF_MODE_AUTO


def test_strerror(lib):
    assert lib.qf_strerror(nat.QF_OK) == b"ok"
    assert lib.qf_strerror(nat.QF_EINVAL) == b"invalid argument"
    assert lib.qf_strerror(12345) == b"unknown status"


def _opts(lib, **kw):
    o = nat.QfOptions()
    lib.qf_options_default(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def test_workspace_size_layout(lib):
    # streaming, complex64: S builders of N^2 complex64 plus one complex128
    # recheck copy each, plus small per-start state
    o = _opts(lib, precision=nat.QF_C64, mode=nat.QF_MODE_STREAMING)
    n, p, S = 10, 45, 16
    N = 1 << n
    ws = lib.qf_workspace_size(n, p, S, ctypes.byref(o))
    assert S * N * N * (8 + 16) <= ws <= S * N * N * (8 + 16) + (8 << 20)
    o = _opts(lib, precision=nat.QF_C128, mode=nat.QF_MODE_STREAMING)
    ws128 = lib.qf_workspace_size(n, p, S, ctypes.byref(o))
    assert S * N * N * 16 <= ws128 <= S * N * N * 16 + (8 << 20)
    # resident mode keeps builders in LDS: small workspace
    o = _opts(lib, mode=nat.QF_MODE_AUTO)
    assert 0 < lib.qf_workspace_size(6, 15, 32, ctypes.byref(o)) < (4 << 20)
    # invalid sizes -> 0
    assert lib.qf_workspace_size(1, 4, 1, None) == 0
    assert lib.qf_workspace_size(17, 4, 1, None) == 0
    assert lib.qf_workspace_size(4, 0, 1, None) == 0
    assert lib.qf_workspace_size(4, 3, 0, None) == 0
    assert lib.qf_workspace_size(4, 3, 1, ctypes.byref(_opts(lib, beta=1.5))) == 0


def test_batch_workspace_size(lib):
    """Batched layout: descriptors, history ring per (block, start), an
    FP64 scratch builder (16 x 16) per hex (16 lanes, one instantiation) of
    the largest launch any shape (8 or 16 hexes per workgroup) can make,
    which the complex128 kernel's fresh FP64 re-evaluations use, and a 4 x 4
    warm-start rotation per (gate, start, half of a sweep)."""
    I32 = ctypes.c_int32
    bn = (I32 * 3)(3, 4, 2)
    go = (I32 * 4)(0, 5, 17, 18)
    o = _opts(lib)
    ws = lib.qf_batch_workspace_size(3, bn, go, 8, ctypes.byref(o))
    ring = o.long_diff_count + 1
    hexes = 2 * 16  # 16 hexes per workgroup hold two blocks of 8 starts: 2 workgroups
    ywarm = 18 * 8 * 2 * 16 * 16
    assert ws >= 3 * 8 * ring * 8 + hexes * 256 * 16 + ywarm
    assert ws <= 3 * 8 * ring * 8 + hexes * 256 * 16 + ywarm + 8192
    # more blocks than a launch has hexes: scratch stops growing
    big = 1 << 16
    bnb = (I32 * big)(*([3] * big))
    gob = (I32 * (big + 1))(*range(big + 1))
    wsb = lib.qf_batch_workspace_size(big, bnb, gob, 1, ctypes.byref(o))
    assert wsb < big * ring * 8 + 32768 * 256 * 16 + big * 2 * 16 * 16 + (4 << 20)
    # invalid -> 0
    assert lib.qf_batch_workspace_size(3, bn, go, 17, ctypes.byref(o)) == 0
    assert lib.qf_batch_workspace_size(3, bn, go, 0, ctypes.byref(o)) == 0
    assert lib.qf_batch_workspace_size(0, bn, go, 8, ctypes.byref(o)) == 0
    bad = (I32 * 3)(3, 5, 2)
    assert lib.qf_batch_workspace_size(3, bad, go, 8, ctypes.byref(o)) == 0
    empty = (I32 * 4)(0, 5, 5, 6)
    assert lib.qf_batch_workspace_size(3, bn, empty, 8, ctypes.byref(o)) == 0


def test_workspace_size3_layout(lib):
    """Three-qubit gates: S builders of N^2 entries (plus an FP64 rebuild
    copy each for complex64), S x p gates of 8 x 8 complex128, their
    warm-start rotations (two 8 x 8 complex128 per gate and start), and
    small per-start state; sizes outside n in [3, 14] are refused."""
    n, p, S = 10, 16, 8
    N = 1 << n
    gates = S * p * 64 * 16 * 3
    o = _opts(lib, precision=nat.QF_C128)
    ws = lib.qf_workspace_size3(n, p, S, ctypes.byref(o))
    assert S * N * N * 16 + gates <= ws <= S * N * N * 16 + gates + (1 << 16)
    o = _opts(lib, precision=nat.QF_C64)
    ws64 = lib.qf_workspace_size3(n, p, S, ctypes.byref(o))
    assert S * N * N * (8 + 16) + gates <= ws64 <= S * N * N * (8 + 16) + gates + (1 << 16)
    assert lib.qf_workspace_size3(3, 1, 1, None) > 0
    assert lib.qf_workspace_size3(2, 1, 1, None) == 0
    assert lib.qf_workspace_size3(15, 1, 1, None) == 0
    assert lib.qf_workspace_size3(5, 0, 1, None) == 0
    assert lib.qf_workspace_size3(5, 2, 0, None) == 0
    assert lib.qf_workspace_size3(5, 2, 1, ctypes.byref(_opts(lib, beta=1.5))) == 0


def test_null_context_is_rejected_before_device_work(lib):
    locs = (ctypes.c_int32 * 2)(0, 1)
    assert lib.qf_instantiate(None, 2, None, 1, locs, None, 1, 1e-8, None, None, 0, None, None, None,
                              None) == nat.QF_EINVAL
    I32 = ctypes.c_int32
    assert lib.qf_instantiate_batch(None, 1, (I32 * 1)(2), (I32 * 2)(0, 1), locs, None, None, 1, 1e-8, None, None,
                                    0, None, None, None, None, None, None) == nat.QF_EINVAL
    assert lib.qf_apply_gate(None, 2, 1, None, 0, locs, None, 0, 0) == nat.QF_EINVAL
    assert lib.qf_environment(None, 2, 1, None, 0, locs, None) == nat.QF_EINVAL
    locs3 = (ctypes.c_int32 * 3)(0, 1, 2)
    assert lib.qf_instantiate3(None, 3, None, 1, locs3, None, 1, 1e-8, None, None, 0, None, None, None,
                               None) == nat.QF_EINVAL
    assert lib.qf_optimize_gate3(None, 1, None, None, 0.0, None) == nat.QF_EINVAL
    assert lib.qf_optimize_gate(None, 1, None, None, 0.0, None) == nat.QF_EINVAL
    assert lib.qf_set_pass2_tiles(None, 1, 10, 4) == nat.QF_EINVAL
    assert lib.qf_destroy(None) == nat.QF_EINVAL
    ctx = ctypes.c_void_p()
    assert lib.qf_create(None, 0, None) == nat.QF_EINVAL
    assert lib.qf_create(ctypes.byref(ctx), -1, None) == nat.QF_EINVAL


def test_package_api_resolves_to_functions():
    for name in ("build", "apply_gate", "environment", "optimize_gate", "update_gate", "cost",
                 "instantiate", "default_options", "workspace_size"):
        assert callable(getattr(pkg, name)), name
    from paper_2306_08152_amd import api
    assert pkg.build is api.build and pkg.instantiate is api.instantiate
    opt = pkg.default_options(precision=1, max_iter=7)
    assert opt.precision == 1 and opt.max_iter == 7 and opt.reset_iter == 40
