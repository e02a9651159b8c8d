"""Pins for the oracle's meshes: counts, the paper's dof counts, geometry,
refinement nesting."""
import numpy as np
import pytest

import fem_inputs
from oracle import mesh as om


@pytest.mark.parametrize("n,p", [(1, 1), (2, 2), (3, 3), (4, 2)])
def test_counts(n, p):
    lev = om.single_level(n, p)
    assert lev.n_cells == 6 * n ** 3
    assert lev.n_dofs == (p * n + 1) ** 3
    assert lev.n_vertices == (n + 1) ** 3
    assert int(lev.interior().sum()) == (p * n - 1) ** 3
    # every lattice point is a node of some cell
    assert np.unique(lev.cell_dofs).size == lev.n_dofs
    # the vertex dofs of each cell are its vertices on the p-lattice
    L = p * n + 1
    vij = lev.cells_ijk * p
    assert np.array_equal(lev.cell_dofs[:, :4], vij[..., 0] + L * (vij[..., 1] + L * vij[..., 2]))


def test_paper_dof_counts():
    # Section 4: P3 on the 32^3 mesh refined twice (128^3) has "about 57 million" dofs,
    # and 111458 dofs per core at 512 processes.
    n_dofs = (3 * 128 + 1) ** 3
    assert n_dofs == 57_066_625
    assert round(n_dofs / 512) == 111_458


@pytest.mark.parametrize("n", [1, 3])
def test_uniform_geometric_factor_closed_form(n):
    # Along the monotone path the Jacobian is a row permutation of h * (upper triangle of ones),
    # so G = |det J| J^-1 J^-T = h [[2,-1,0],[-1,2,-1],[0,-1,1]] for every cell.
    lev = om.single_level(n, 1)
    G, det = lev.geometric_factors()
    h = 1.0 / n
    expect = h * np.array([[2.0, -1.0, 0.0], [-1.0, 2.0, -1.0], [0.0, -1.0, 1.0]])
    assert np.max(np.abs(G - expect)) < 1e-14
    assert np.allclose(det, h ** 3, rtol=1e-14)


@pytest.mark.parametrize("jit", [False, True])
def test_volume_and_validity(jit):
    n = 4
    j = fem_inputs.jitter_offsets(n, 0.15) if jit else None
    levels = om.hierarchy(n, 2, 1, j)
    for lev in levels:
        _, det = lev.geometric_factors()
        assert det.min() > 0.2 * lev.h ** 3
        assert abs(det.sum() / 6.0 - 1.0) < 1e-13


@pytest.mark.parametrize("jit", [False, True])
def test_refinement_nesting(jit):
    n = 2
    j = fem_inputs.jitter_offsets(n, 0.15) if jit else None
    coarse, fine = om.hierarchy(n, 1, 1, j)
    xc = coarse.cell_xyz()
    Jc = np.stack([xc[:, 1] - xc[:, 0], xc[:, 2] - xc[:, 0], xc[:, 3] - xc[:, 0]], axis=2)
    Jinv = np.linalg.inv(Jc)
    xf = fine.cell_xyz()
    parents = []
    for c in range(fine.n_cells):
        # barycentric coordinates of all 4 fine vertices in every coarse cell
        loc = np.einsum("cij,cvj->cvi", Jinv, xf[c][None, :, :] - xc[:, 0][:, None, :])
        lam = np.concatenate([1.0 - loc.sum(axis=2, keepdims=True), loc], axis=2)
        inside = np.all(lam > -1e-12, axis=(1, 2))
        assert inside.sum() == 1, "each fine cell lies in exactly one coarse cell"
        parents.append(int(np.argmax(inside)))
    counts = np.bincount(parents, minlength=coarse.n_cells)
    assert np.all(counts == 8)


def test_refined_vertices_are_midpoints():
    n = 2
    j = fem_inputs.jitter_offsets(n, 0.15)
    coarse, fine = om.hierarchy(n, 1, 1, j)
    # coarse vertices are kept
    ijk = fem_inputs.vertex_lattice(n)
    assert np.array_equal(fine.vert_xyz[om.vertex_id(2 * n, 2 * ijk)], coarse.vert_xyz)


def test_dof_positions_consistent():
    lev = om.single_level(3, 3)
    xyz = lev.dof_xyz()
    lat = om.dof_lattice(3, 3)
    assert np.allclose(xyz, lat / 9.0, atol=1e-15)
