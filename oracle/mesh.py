"""Tetrahedral unit-cube meshes, their uniform refinement and P_p numbering.

Follows Section 2, Listing 1 of the paper: UnitCubeMesh(N, N, N) and
MeshHierarchy(mesh, 2), i.e. a tetrahedral unit cube refined uniformly.

Readings of the paper taken here:
* Each of the n^3 cubes is split into the 6 tetrahedra that share its main
  diagonal (Kuhn / Freudenthal split).  For the axis permutation s the cell's
  vertices follow the monotone lattice path
      v0 = c, v1 = v0 + e_s0, v2 = v1 + e_s1, v3 = c + (1,1,1),
  c the cube's lower corner.  This split reproduces the paper's degree-of-
  freedom counts ((p n + 1)^3 total; Section 4 quotes about 57 million for P3
  on 128^3, which is 385^3).
* Uniform refinement puts the new vertices at edge midpoints; refining the
  split of n^3 cubes gives exactly the split of (2n)^3 cubes, with every fine
  cell inside one coarse cell.
* Jittered variant: only the coarsest level's interior vertices move; every
  finer vertex is the midpoint of the coarse edge it refines, so the meshes
  stay nested.

P_p degrees of freedom sit on the lattice of spacing h/p: the node with
barycentric multi-index m in a cell with integer vertex coordinates V_i has
lattice coordinates sum_i m_i V_i.  Global dof id = I + L (J + L K) with
L = p n + 1.  Boundary dofs are those with a lattice coordinate equal to 0 or
p n.

Parity: counts, nesting and the geometric factors of the uniform mesh are
pinned in tests/test_oracle_mesh.py.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from itertools import permutations

import numpy as np

from . import refelem

PERMS = tuple(permutations(range(3)))  # 6 axis orders, one tetrahedron each


def kuhn_cells(n: int) -> np.ndarray:
    """Integer vertex coordinates of all cells: (6 n^3, 4, 3), cube-major."""
    r = np.arange(n)
    kk, jj, ii = np.meshgrid(r, r, r, indexing="ij")
    corners = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1)  # (n^3, 3)
    return cube_cells(corners)


def cube_cells(corners: np.ndarray) -> np.ndarray:
    """The 6 tetrahedra of each cube with the given lower corners: (6 m, 4, 3), cube-major."""
    corners = np.asarray(corners, dtype=np.int64).reshape(-1, 3)
    cells = np.zeros((corners.shape[0], 6, 4, 3), dtype=np.int64)
    for t, s in enumerate(PERMS):
        v = corners.copy()
        cells[:, t, 0] = v
        v = v.copy()
        v[:, s[0]] += 1
        cells[:, t, 1] = v
        v = v.copy()
        v[:, s[1]] += 1
        cells[:, t, 2] = v
        cells[:, t, 3] = corners + 1
    return cells.reshape(-1, 4, 3)


def vertex_id(n: int, ijk: np.ndarray) -> np.ndarray:
    ijk = np.asarray(ijk)
    return ijk[..., 0] + (n + 1) * (ijk[..., 1] + (n + 1) * ijk[..., 2])


def dof_lattice(n: int, p: int) -> np.ndarray:
    """Lattice coordinates of every dof, (L^3, 3), x fastest."""
    L = p * n + 1
    r = np.arange(L)
    k, j, i = np.meshgrid(r, r, r, indexing="ij")
    return np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)


@dataclass
class Level:
    n: int
    p: int
    cells_ijk: np.ndarray        # (C, 4, 3) integer vertex coordinates
    vert_xyz: np.ndarray         # ((n+1)^3, 3) vertex positions
    cell_vert: np.ndarray = field(init=False)   # (C, 4) vertex ids
    cell_dofs: np.ndarray = field(init=False)   # (C, nloc) dof ids
    n_dofs: int = field(init=False)
    n_vertices: int = field(init=False)
    boundary: np.ndarray = field(init=False)    # (n_dofs,) bool

    def __post_init__(self):
        n, p = self.n, self.p
        L = p * n + 1
        self.n_dofs = L ** 3
        self.n_vertices = (n + 1) ** 3
        self.cell_vert = vertex_id(n, self.cells_ijk)
        mi = np.array(refelem.node_multi_indices(p), dtype=np.int64)      # (nloc, 4)
        lat = np.einsum("li,cid->cld", mi, self.cells_ijk)                  # (C, nloc, 3)
        self.cell_dofs = lat[..., 0] + L * (lat[..., 1] + L * lat[..., 2])
        lattice = dof_lattice(n, p)
        self.boundary = np.any((lattice == 0) | (lattice == p * n), axis=1)

    @property
    def n_cells(self) -> int:
        return self.cells_ijk.shape[0]

    @property
    def h(self) -> float:
        return 1.0 / self.n

    def cell_xyz(self) -> np.ndarray:
        """Vertex positions per cell, (C, 4, 3)."""
        return self.vert_xyz[self.cell_vert]

    def jacobians(self) -> np.ndarray:
        """J = [x1-x0 | x2-x0 | x3-x0] per cell, (C, 3, 3) (columns are edges)."""
        x = self.cell_xyz()
        return np.stack([x[:, 1] - x[:, 0], x[:, 2] - x[:, 0], x[:, 3] - x[:, 0]], axis=2)

    def geometric_factors(self):
        """(G, |det J|) with G = |det J| J^-1 J^-T, per cell."""
        J = self.jacobians()
        det = np.linalg.det(J)
        Jinv = np.linalg.inv(J)
        G = np.abs(det)[:, None, None] * np.einsum("cai,cbi->cab", Jinv, Jinv)
        return G, np.abs(det)

    def dof_xyz(self) -> np.ndarray:
        """Physical position of each dof, (n_dofs, 3)."""
        mi = np.array(refelem.node_multi_indices(self.p), dtype=np.float64) / self.p
        pos = np.einsum("li,cid->cld", mi, self.cell_xyz())
        out = np.zeros((self.n_dofs, 3))
        out[self.cell_dofs.ravel()] = pos.reshape(-1, 3)
        return out

    def interior(self) -> np.ndarray:
        return ~self.boundary


def uniform_vertices(n: int) -> np.ndarray:
    r = np.arange(n + 1, dtype=np.float64) / n
    k, j, i = np.meshgrid(r, r, r, indexing="ij")
    return np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)


def refine_vertices(n: int, coarse_xyz: np.ndarray) -> np.ndarray:
    """Vertex positions of the refined mesh (2n): coarse vertices stay, new
    vertices are midpoints of the coarse edges they split."""
    ijk = dof_lattice(2 * n, 1)                     # fine vertex lattice = P1 on 2n
    lo = ijk // 2
    hi = (ijk + 1) // 2
    return 0.5 * (coarse_xyz[vertex_id(n, lo)] + coarse_xyz[vertex_id(n, hi)])


def hierarchy(n0: int, n_refine: int, p: int, jitter: np.ndarray | None = None):
    """Levels coarsest-first.  jitter: ((n0+1)^3, 3) offsets in units of h0."""
    xyz = uniform_vertices(n0)
    if jitter is not None:
        xyz = xyz + np.asarray(jitter, dtype=np.float64) / n0
    levels = []
    n = n0
    for ell in range(n_refine + 1):
        if ell > 0:
            xyz = refine_vertices(n, xyz)
            n *= 2
        levels.append(Level(n=n, p=p, cells_ijk=kuhn_cells(n), vert_xyz=xyz))
    return levels


def single_level(n: int, p: int, jitter: np.ndarray | None = None) -> Level:
    return hierarchy(n, 0, p, jitter)[0]
