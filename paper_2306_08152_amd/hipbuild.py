"""Build the HIP library (gfx950) in-tree: paper_2306_08152_amd/lib/libqfactor_mi355x.so.

Usage: python -m paper_2306_08152_amd.hipbuild  (or call build()).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIBDIR = os.path.join(PKG, "lib")
LIBNAME = "libqfactor_mi355x.so"
SOURCES = ["qf_stream.hip", "qf_pair.hip", "qf_resident.hip", "qf_batch.hip", "qf_grad.hip", "qf_k3.hip",
           "qf_abi.hip"]
ARCH = "gfx950"

# Packed FP32 instructions are switched off for every HIP translation unit.
HIP_FLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


# Host-side AddressSanitizer + UndefinedBehaviorSanitizer build of the same
# sources (device code unchanged): each -fsanitize= applies to the host pass
# only.  Loaded in a process that preloads the ASan runtime; see
# tests/test_sanitized_host.py.
SANITIZE_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
SANITIZED_LIBNAME = "libqfactor_mi355x_asan.so"


def lib_path() -> str:
    """Path of the library the binding loads: the environment variable
    QF_LIBRARY when set (the sanitized build in its test), else the in-tree
    build."""
    return os.environ.get("QF_LIBRARY") or os.path.join(LIBDIR, LIBNAME)


def sanitized_lib_path() -> str:
    return os.path.join(LIBDIR, SANITIZED_LIBNAME)


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found; the HIP library cannot be built")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return r


def build(verbose: bool = False, jobs: int = 3, sanitize: bool = False) -> str:
    """Compile every source for gfx950 and link the shared library.  Always
    rebuilds.  sanitize=True builds the host-sanitized variant instead
    (sanitized_lib_path()).  Returns the library path."""
    cc = hipcc()
    os.makedirs(LIBDIR, exist_ok=True)
    objdir = os.path.join(PKG, "_build_asan" if sanitize else "_build")
    os.makedirs(objdir, exist_ok=True)
    inc = ["-I", INCLUDE, "-I", CSRC]
    extra = SANITIZE_FLAGS if sanitize else []
    objs = []
    cmds = []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        objs.append(obj)
        cmds.append([cc, *HIP_FLAGS, *extra, *inc, "-c", os.path.join(CSRC, src), "-o", obj])
    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        list(ex.map(lambda c: _run(c, verbose), cmds))
    out = sanitized_lib_path() if sanitize else os.path.join(LIBDIR, LIBNAME)
    tmp = out + ".tmp"
    _run([cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *extra, *objs, "-o", tmp], verbose)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
