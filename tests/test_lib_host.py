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


def test_solver_workspace_coarse_choices():
    """Coarse-level choice: dense inverse up to 40000 interior dofs, nested MG-PCG above (or on
    request), and an error where neither applies."""
    import ctypes as C
    from paper_2104_08012_amd import fem
    from paper_2104_08012_amd import _lib as L
    m = fem.Mesh(2, 4, 2, upload=False)        # P2 on 2^3 .. 32^3 cubes; 32^3 has 63^3 interior dofs

    def ws(**kw):
        o, keep, _ = fem.SolveOptions(**kw).to_c()
        nb = C.c_size_t()
        st = L.lib().fem_solve_workspace_bytes(m.handle, C.byref(o), C.byref(nb))
        return st, nb.value

    st_d, b_d = ws()                                            # dense on level 0 (27 interior)
    assert st_d == 0 and b_d % 256 == 0
    st, _ = ws(n_levels_used=1, coarse_method="dense")          # 250047 interior: too large
    assert st == L.FEM_ERR_UNSUPPORTED
    st_n, b_n = ws(n_levels_used=1)                             # auto -> nested over levels 0..4
    assert st_n == 0
    st_n2, b_n2 = ws(n_levels_used=1, coarse_method="nested")
    assert st_n2 == 0 and b_n2 == b_n
    # nested: vectors of the levels plus the dense inverse of the 8^3 level (3375 interior dofs,
    # the finest level with at most 8000), never a dense 250047^2 block
    n4 = m.levels[4]["n_dofs"]
    assert 4 * n4 * 8 + 3375 ** 2 * 8 < b_n < 64 * n4 * 8 + 3 * 3375 ** 2 * 8
    st, _ = ws(coarse_method="nested")                          # nothing below level 0
    assert st == L.FEM_ERR_UNSUPPORTED
    st_m, b_m = ws(n_levels_used=2, precision="mixed")          # 16^3 coarse: dense, 31^3 dofs
    assert st_m == 0 and b_m > 31 ** 6 * 8
    # the mixed solver keeps the FP64 coarse inverse: its packed half-matrix tiles take at least
    # 31^6 / 2 * 8 bytes beside the 31^6 * 8 of the dense block; the FP32-stored inverse is an
    # explicit option that halves them, and is refused in FP64
    assert b_m > 31 ** 6 * 8 + 31 ** 6 * 4
    st_f, b_f = ws(n_levels_used=2, precision="mixed", coarse_method="dense_f32")
    assert st_f == 0 and b_m - b_f > 31 ** 6 * 2 * 0.9
    st, _ = ws(n_levels_used=2, coarse_method="dense_f32")
    assert st == L.FEM_ERR_INVALID_ARG


@pytest.mark.parametrize("n,p", [(3, 1), (2, 2), (2, 3), (4, 2)])
def test_csr_pattern_matches_oracle(n, p):
    """The host CSR pattern equals the sparsity of the oracle's assembled stiffness matrix (the
    union of the cells' dof couplings), row by row in the library's (lattice) dof order."""
    import scipy.sparse as sp
    from paper_2104_08012_amd import fem
    from oracle import assemble
    from oracle import mesh as om
    m = fem.Mesh(n, 0, p, upload=False)
    A = fem.CsrOperator(m, 0, upload=False)
    rp, col = A.pattern()
    lev = om.single_level(n, p)
    S = sp.csr_matrix(assemble.stiffness(lev))
    S.sort_indices()
    assert A.n_rows == lev.n_dofs and A.nnz == S.nnz
    assert np.array_equal(rp, S.indptr) and np.array_equal(col, S.indices)


def test_patch_buffer_bytes_and_degree_check():
    import ctypes as C
    from paper_2104_08012_amd import fem
    from paper_2104_08012_amd._lib import FEM_ERR_UNSUPPORTED, FEM_OK, lib

    def a256(x):
        return (x + 255) // 256 * 256

    def pad64(x):   # the per-vertex entries are stored in blocks of 64 vertices
        return (x + 63) // 64 * 64

    m = fem.Mesh(6, 1, 2, upload=False)
    nb = C.c_size_t()
    for level, n in ((0, 6), (1, 12)):
        NV = pad64((n + 1) ** 3)
        for dt, s in ((0, 8), (1, 4)):
            assert lib().fem_patch_bytes(m.handle, level, dt, C.byref(nb)) == FEM_OK
            assert nb.value == a256(120 * NV * s) + a256(15 * NV * s)
    m3 = fem.Mesh(3, 1, 3, upload=False)           # P3 stars: 2145 packed entries + 65 results
    for level, n in ((0, 3), (1, 6)):
        NV = pad64((n + 1) ** 3)
        for dt, s in ((0, 8), (1, 4)):
            assert lib().fem_patch_bytes(m3.handle, level, dt, C.byref(nb)) == FEM_OK
            assert nb.value == a256(2145 * NV * s) + a256(65 * NV * s)
    mp = fem.Mesh(2, 0, 1, upload=False)           # P1: every star is one dof (Jacobi)
    assert lib().fem_patch_bytes(mp.handle, 0, 0, C.byref(nb)) == FEM_ERR_UNSUPPORTED
    # the packed star index is 32-bit: (2145 + 65) * n_vertices must stay below 2^32, which P3
    # at 128^3 cubes (2,146,689 vertices) exceeds
    big = fem.Mesh(128, 0, 3, upload=False)
    assert lib().fem_patch_bytes(big.handle, 0, 0, C.byref(nb)) == FEM_ERR_UNSUPPORTED
    assert lib().fem_patch_bytes(m.handle, 2, 0, C.byref(nb)) != FEM_OK


def test_solver_workspace_with_patch_smoother():
    """The star-patch smoother adds, per smoothed level, the patch buffer (120 + 15 entries per
    vertex for P2, 2145 + 65 for P3, the vertex count rounded up to a multiple of 64) and one level
    vector; degree 1 is refused."""
    import ctypes as C
    from paper_2104_08012_amd import fem
    from paper_2104_08012_amd import _lib as L

    def ws(m, **kw):
        o, keep, _ = fem.SolveOptions(**kw).to_c()
        nb = C.c_size_t()
        st = L.lib().fem_solve_workspace_bytes(m.handle, C.byref(o), C.byref(nb))
        return st, nb.value

    m = fem.Mesh(4, 2, 2, upload=False)
    for prec, s in (("fp64", 8), ("mixed", 4)):
        st_j, b_j = ws(m, precision=prec)
        st_p, b_p = ws(m, precision=prec, smoother="patch")
        assert st_j == 0 and st_p == 0
        extra = sum(135 * ((m.levels[l]["n_vertices"] + 63) // 64 * 64) * s + m.levels[l]["n_dofs"] * s
                    for l in (1, 2))
        assert extra <= b_p - b_j <= extra + 6 * 256
    m3 = fem.Mesh(2, 2, 3, upload=False)
    for prec, s in (("fp64", 8), ("mixed", 4)):
        st_j, b_j = ws(m3, precision=prec)
        st_p, b_p = ws(m3, precision=prec, smoother="patch")
        assert st_j == 0 and st_p == 0
        extra = sum(2210 * ((m3.levels[l]["n_vertices"] + 63) // 64 * 64) * s + m3.levels[l]["n_dofs"] * s
                    for l in (1, 2))
        assert extra <= b_p - b_j <= extra + 6 * 256
    mp = fem.Mesh(2, 1, 1, upload=False)
    st, _ = ws(mp, smoother="patch")
    assert st == L.FEM_ERR_UNSUPPORTED


def test_action_geometry_source_per_level():
    """Levels on 4-cube bricks take G from the coarsest level's table once a brick lies in one
    coarsest cube (level >= 2, coarsest mesh up to 24^3); before that P1/P2 form it from the vertex
    coordinates and P3 reads per-cell factors, as every level on smaller bricks does.  (The library
    checks the table against every cell's factors when it builds the mesh.)"""
    from paper_2104_08012_amd import fem
    m = fem.Mesh(4, 3, 2, upload=False)
    assert [m.info(l)["geometry"] for l in range(4)] == ["vertex", "vertex", "table", "table"]
    m = fem.Mesh(3, 2, 1, jitter=fem_inputs.jitter_offsets(3, 0.15), upload=False)
    assert [m.info(l)["geometry"] for l in range(3)] == ["cell", "cell", "table"]   # n = 3, 6: bricks of 1, 2
    assert fem.Mesh(32, 0, 2, upload=False).info(0)["geometry"] == "vertex"
    assert fem.Mesh(28, 2, 1, upload=False).info(2)["geometry"] == "vertex"       # coarsest above 24^3
    m = fem.Mesh(2, 2, 3, upload=False)
    assert [m.info(l)["geometry"] for l in range(3)] == ["cell", "cell", "table"]
    assert fem.Mesh(8, 0, 3, upload=False).info(0)["geometry"] == "cell"
