"""The kernels' compile-time quadrature tabulations agree with the host rules (which are checked
for exactness against the monomial moments at library start) to 1e-14."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_compile_time_tabulation_matches_host_rules():
    src = os.path.join(ROOT, "tests", "tab_check.cpp")
    ref = os.path.join(ROOT, "paper_2104_08012_amd", "csrc", "refelem.cpp")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "tab_check")
        subprocess.run(["g++", "-O1", "-std=c++17", "-I", os.path.join(ROOT, "include"), src, ref, "-o", exe],
                       check=True, capture_output=True)
        r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert float(r.stdout.strip()) < 1e-14
