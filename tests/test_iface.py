"""The per-face affine numbering of interface slots (the cube kernel's write-out) equals the
point-wise numbering, stays inside the slot array and gives every (brick, face point) pair its own
slot, for brick spans PB = 1, 2, 3, 4, 8, 12 and 1-5 bricks per direction."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_affine_interface_numbering():
    src = os.path.join(ROOT, "tests", "iface_check.cpp")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "iface_check")
        subprocess.run(["g++", "-O1", "-std=c++17", src, "-o", exe], check=True, capture_output=True)
        r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip() == "0"
