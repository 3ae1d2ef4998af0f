"""The C ABI's host logic under AddressSanitizer and UndefinedBehaviorSanitizer.

The library is rebuilt with host-side sanitizers (device code unchanged,
paper_2306_08152_amd.hipbuild.build(sanitize=True)) and tests/test_abi_host.py
runs against it in a child process that preloads the ASan runtime: argument
validation, workspace layouts, option defaults and error strings are
exercised with bounds, use-after-free and undefined-behaviour checks on.  No
GPU is used (the host paths under test stop before any device call)."""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan_runtime():
    cands = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return cands[-1] if cands else None


def test_abi_host_under_asan_and_ubsan():
    rt = _asan_runtime()
    if rt is None or not (os.path.exists("/opt/rocm/bin/hipcc") or shutil.which("hipcc")):
        pytest.skip("hipcc or the ASan runtime is not available")
    sys.path.insert(0, ROOT)
    from paper_2306_08152_amd.hipbuild import build
    lib = build(sanitize=True, jobs=4)
    env = dict(os.environ, QF_LIBRARY=lib, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    # the build is instrumented (it calls the ASan and UBSan runtimes), and
    # the child process loads it with the runtime present
    with open(lib, "rb") as f:
        image = f.read()
    assert b"__asan_report_load8" in image and b"__ubsan_handle" in image
    probe = ("import ctypes, paper_2306_08152_amd._native as n; l = n.load(); "
             "print(l._name); ctypes.CDLL(None).__asan_report_load8")
    r = subprocess.run([sys.executable, "-c", probe], env=env, cwd=ROOT, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip().endswith("libqfactor_mi355x_asan.so"), r.stdout + r.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi_host.py")],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
