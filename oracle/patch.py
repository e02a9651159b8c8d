"""Additive vertex-star patch preconditioner (test infrastructure only).

Only tests/, the smoke check and the benchmark's CPU baseline use this module;
the library never calls it.

Follows Section 2, Listing 2: the multigrid smoother's preconditioner is the
patch preconditioner with star patches built around mesh vertices
(construct_type star, construct_dim 0), combined additively.  Definition:

* The patch of vertex v holds the degrees of freedom carried by the mesh
  entities whose closure contains v (v itself and the edges, faces and cells
  incident to it).  In a cell where v is local vertex i, the node with
  barycentric multi-index m belongs to that entity set exactly when m_i > 0.
* Dirichlet (boundary) dofs belong to no patch.
* With R_v the restriction to the patch and A_v = R_v A R_v^T,
      z = sum_v R_v^T A_v^{-1} R_v r      on interior dofs.

Reading of the paper taken here: the system matrix carries identity rows for the
boundary dofs; the preconditioner passes those entries through, z_B = r_B
(each boundary dof acts as a patch of its own with matrix 1).

Pins (tests/test_oracle_patch.py): for P1 every star holds one dof, so the
preconditioner is point Jacobi; the star sizes of an interior vertex follow
from the link of a vertex in the cube split (14 vertices, 36 edges, 24
triangles); with A = I every dof is counted once per vertex of the entity that
carries it; patch matrices equal the sum of the element matrices of the cells
around v; the preconditioner is symmetric positive definite.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import refelem
from .mesh import Level


def star_patches(level: Level) -> list[np.ndarray]:
    """Interior dof ids of every vertex star, indexed by vertex id (sorted, possibly empty)."""
    mi = np.array(refelem.node_multi_indices(level.p), dtype=np.int64)   # (nloc, 4)
    verts, dofs = [], []
    for i in range(4):
        sel = mi[:, i] > 0
        d = level.cell_dofs[:, sel]                                         # (C, ns)
        verts.append(np.repeat(level.cell_vert[:, i], d.shape[1]))
        dofs.append(d.ravel())
    verts = np.concatenate(verts)
    dofs = np.concatenate(dofs)
    keep = ~level.boundary[dofs]
    pairs = np.unique(np.stack([verts[keep], dofs[keep]], axis=1), axis=0)
    out = [np.zeros(0, dtype=np.int64) for _ in range(level.n_vertices)]
    if pairs.size:
        starts = np.searchsorted(pairs[:, 0], np.arange(level.n_vertices + 1))
        for v in range(level.n_vertices):
            out[v] = pairs[starts[v]:starts[v + 1], 1]
    return out


def patch_inverses(A: sp.csr_matrix, patches: list[np.ndarray]) -> list[np.ndarray]:
    """A_v^{-1} for every patch (dense), A_v the principal submatrix of A on the patch."""
    A = sp.csr_matrix(A)
    return [np.linalg.inv(A[idx][:, idx].toarray()) if idx.size else np.zeros((0, 0)) for idx in patches]


def apply_patch_pc(patches: list[np.ndarray], inverses: list[np.ndarray], boundary: np.ndarray,
                   r: np.ndarray) -> np.ndarray:
    """z = sum_v R_v^T A_v^{-1} R_v r on interior dofs, z_B = r_B."""
    r = np.asarray(r, dtype=np.float64)
    z = np.zeros_like(r)
    z[boundary] = r[boundary]
    for idx, inv in zip(patches, inverses):
        if idx.size:
            z[idx] += inv @ r[idx]
    return z


def patch_pc_at(level: Level, k_vertex, r: np.ndarray, dofs) -> np.ndarray:
    """z = B_patch r at the given dofs only, for meshes too large for the global construction:
    every star containing a dof is assembled from the element matrices of the cells around its
    vertex (the cells coupling two dofs of a star all contain its vertex, so this is the
    principal submatrix of the global operator on the star) and solved densely."""
    from . import assemble
    mi = np.array(refelem.node_multi_indices(level.p), dtype=np.int64)
    r = np.asarray(r, dtype=np.float64)
    out = np.empty(len(dofs))
    for j, g in enumerate(dofs):
        g = int(g)
        if level.boundary[g]:
            out[j] = r[g]
            continue
        c, a = (int(t[0]) for t in np.nonzero(level.cell_dofs == g))
        total = 0.0
        for v in level.cell_vert[c, mi[a] > 0]:
            cells = np.nonzero((level.cell_vert == v).any(axis=1))[0]
            Ae = assemble.element_matrices(level, k_vertex, cells)
            iv = np.argmax(level.cell_vert[cells] == v, axis=1)
            rows, cols, vals = [], [], []
            for q, cc in enumerate(cells):
                loc = np.nonzero(mi[:, iv[q]] > 0)[0]
                d = level.cell_dofs[cc, loc]
                rows.append(np.repeat(d, loc.size))
                cols.append(np.tile(d, loc.size))
                vals.append(Ae[q][np.ix_(loc, loc)].ravel())
            rows, cols, vals = np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
            keep = ~level.boundary[rows] & ~level.boundary[cols]
            star = np.unique(rows[keep])
            pos = {int(d): i for i, d in enumerate(star)}
            Av = np.zeros((star.size, star.size))
            np.add.at(Av, (np.array([pos[int(d)] for d in rows[keep]]),
                           np.array([pos[int(d)] for d in cols[keep]])), vals[keep])
            total += np.linalg.solve(Av, r[star])[pos[g]]
        out[j] = total
    return out
