"""Interface numbering (iface.hpp): the per-face affine indices equal the point-wise numbering,
stay inside the slot array and give every (brick, face point) pair its own slot, for cubic bricks
(span 1-12, 1-5 per direction) and bricks merged along x (span 2-4 PB); and the merged-brick
write-out regions of the cube kernel write every non-interface point to y exactly once and every
(brick, interface point) slot exactly once."""
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
