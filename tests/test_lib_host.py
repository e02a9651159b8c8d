"""CPU checks of the HIP library: it loads, exports every symbol of include/fem.h, and its
host-side mesh construction agrees with the oracle's (counts, lattice, vertex positions).
No kernel is launched here."""
import ctypes
import os
import re

import numpy as np
import pytest

import fem_inputs
from oracle import mesh as om

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "fem.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(fem_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    from paper_2104_08012_amd import _lib
    L = ctypes.CDLL(_lib.LIB_PATH)
    names = _declared_symbols()
    assert len(names) >= 20
    for name in names:
        assert hasattr(L, name), name
    # the Python binding declares the same set
    assert set(names) == set(_lib.SIGNATURES)


@pytest.mark.parametrize("n,r,p,jit", [(3, 1, 3, 0.15), (4, 2, 2, 0.0), (2, 2, 1, 0.1), (5, 0, 2, 0.15)])
def test_host_mesh_matches_oracle(n, r, p, jit):
    from paper_2104_08012_amd import fem
    j = fem_inputs.jitter_offsets(n, jit) if jit else None
    m = fem.Mesh(n, r, p, jitter=j, upload=False)
    levels = om.hierarchy(n, r, p, j)
    assert m.n_levels == r + 1
    for ell, lev in enumerate(levels):
        info = m.info(ell)
        assert info["n_cells"] == lev.n_cells
        assert info["n_dofs"] == lev.n_dofs
        assert info["n_vertices"] == lev.n_vertices
        assert info["n_interior"] == int(lev.interior().sum())
        assert np.array_equal(m.dof_lattice(ell), om.dof_lattice(lev.n, p))
        assert np.max(np.abs(m.vertex_coords(ell) - lev.vert_xyz)) < 1e-15
        assert info["brick"] in (1, 2, 4) and lev.n % info["brick"] == 0


def test_invalid_mesh_arguments():
    from paper_2104_08012_amd import fem
    from paper_2104_08012_amd._lib import FemError
    with pytest.raises(FemError):
        fem.Mesh(0, 0, 2, upload=False)
    with pytest.raises(FemError):
        fem.Mesh(2, 0, 4, upload=False)
    with pytest.raises(FemError):
        fem.Mesh(2, 9, 1, upload=False)
    big = fem_inputs.jitter_offsets(2, 0.0)
    big[13] = [0.95, -0.95, 0.0]   # the centre vertex of Kuhn(2) pushed far enough to invert cells
    with pytest.raises(FemError, match="inverted"):
        fem.Mesh(2, 0, 1, jitter=big, upload=False)


def test_mesh_device_bytes_scale():
    from paper_2104_08012_amd import fem
    m = fem.Mesh(8, 0, 2, upload=False)
    b = m.device_bytes()
    C = 6 * 8 ** 3
    # map (10 int32), G (6 f64 + 6 f32) per cell at least
    assert b >= C * (10 * 4 + 6 * 12) and b % 256 == 0
