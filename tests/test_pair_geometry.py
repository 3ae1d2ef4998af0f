"""Host check of the index maps of the two-gate pass and environment
(paper_2306_08152_amd/csrc/qf_pair_geom.h): tests/native/pair_geom_check.cpp,
built for the host, enumerates every tile geometry of every gate pair that
forms a 3- or 4-qubit union (all pairs up to n = 8, a sample at n = 9) in
both builder precisions and checks that the address-order phases move every
builder entry exactly once, that each tile's LDS image holds the entries the
product phases assume, and that each gate's phase covers the tile with 4x4
blocks varying only in that gate's bits.  No GPU is used."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _compiler():
    for c in ("/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    return None


def test_pair_geometry_covers_every_entry_once(tmp_path):
    cc = _compiler()
    if cc is None:
        pytest.skip("hipcc not available")
    exe = tmp_path / "pair_geom_check"
    src = os.path.join(ROOT, "tests", "native", "pair_geom_check.cpp")
    inc = os.path.join(ROOT, "paper_2306_08152_amd", "csrc")
    subprocess.run([cc, "-O2", "-std=c++17", "-I", inc, src, "-o", str(exe)], check=True, capture_output=True)
    r = subprocess.run([str(exe), "9"], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok"), r.stdout
    assert int(r.stdout.split()[1]) > 5000
