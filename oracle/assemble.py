"""Assembled and matrix-free FP64 operators: stiffness -div(k grad u), mass.

Follows the weak form of Section 2, eq. (4): a(u, v) = int k grad(u).grad(v),
with k = 1 (the paper's case) or k a P1 field given by its vertex values.
Element matrices come from the exact reference tensors (refelem):

  constant k:  A_K = sum_ab G_ab S^{ab}
  P1 k:        A_K = sum_v k_v sum_ab G_ab T^{v,ab}
  mass:        M_K = |det J| M_ref

with G = |det J| J^-1 J^-T.  Dirichlet conditions on all six faces
(Listing 1's DirichletBC) by symmetric elimination:
  A_bc = P_I A P_I + P_B   (identity rows and zero columns on boundary dofs).

Parity: the assembled operator is pinned by closed forms (P1 on the uniform
split is h times the 7-point finite-difference Laplacian), exact
reproduction of linear/quadratic/cubic fields and A.1 = 0, and, for the P1
coefficient, exact reproduction of -div(ell grad q) with ell linear (which
fails if the vertex weights of T^{v,ab} are permuted), in
tests/test_oracle_assembly.py.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import refelem
from .mesh import Level


def element_matrices(level: Level, k_vertex: np.ndarray | None = None,
                     cells: slice | np.ndarray | None = None) -> np.ndarray:
    """Element stiffness matrices (C, nloc, nloc) for a subset of cells."""
    G, _ = level.geometric_factors() if cells is None else _gf_subset(level, cells)
    p = level.p
    if k_vertex is None:
        return np.einsum("cab,abij->cij", G, refelem.S(p))
    cv = level.cell_vert if cells is None else level.cell_vert[cells]
    kc = np.asarray(k_vertex, dtype=np.float64)[cv]                     # (C, 4)
    return np.einsum("cv,cab,vabij->cij", kc, G, refelem.T(p))


def _gf_subset(level: Level, cells):
    x = level.vert_xyz[level.cell_vert[cells]]
    J = np.stack([x[:, 1] - x[:, 0], x[:, 2] - x[:, 0], x[:, 3] - x[:, 0]], axis=2)
    det = np.linalg.det(J)
    Jinv = np.linalg.inv(J)
    G = np.abs(det)[:, None, None] * np.einsum("cai,cbi->cab", Jinv, Jinv)
    return G, np.abs(det)


def mass_element_matrices(level: Level) -> np.ndarray:
    _, det = level.geometric_factors()
    return det[:, None, None] * refelem.M(level.p)[None]


def _assemble(level: Level, Ae: np.ndarray) -> sp.csr_matrix:
    dofs = level.cell_dofs
    nl = dofs.shape[1]
    rows = np.repeat(dofs, nl, axis=1).ravel()
    cols = np.tile(dofs, (1, nl)).ravel()
    A = sp.coo_matrix((Ae.ravel(), (rows, cols)), shape=(level.n_dofs, level.n_dofs))
    return A.tocsr()


def stiffness(level: Level, k_vertex: np.ndarray | None = None, chunk: int = 1 << 18) -> sp.csr_matrix:
    """Raw assembled stiffness matrix (no boundary conditions), CSR."""
    C = level.n_cells
    if C <= chunk:
        return _assemble(level, element_matrices(level, k_vertex))
    A = None
    for s in range(0, C, chunk):
        sl = slice(s, min(C, s + chunk))
        Ae = element_matrices(level, k_vertex, sl)
        dofs = level.cell_dofs[sl]
        nl = dofs.shape[1]
        rows = np.repeat(dofs, nl, axis=1).ravel()
        cols = np.tile(dofs, (1, nl)).ravel()
        part = sp.coo_matrix((Ae.ravel(), (rows, cols)), shape=(level.n_dofs, level.n_dofs)).tocsr()
        A = part if A is None else A + part
    return A


def mass(level: Level) -> sp.csr_matrix:
    return _assemble(level, mass_element_matrices(level))


def apply_bc(A: sp.csr_matrix, boundary: np.ndarray) -> sp.csr_matrix:
    """Symmetric elimination: A_bc = P_I A P_I + P_B."""
    interior = (~boundary).astype(np.float64)
    PI = sp.diags(interior)
    PB = sp.diags(boundary.astype(np.float64))
    return (PI @ A @ PI + PB).tocsr()


def matfree_action(level: Level, x: np.ndarray, k_vertex: np.ndarray | None = None,
                   bc: bool = True, chunk: int = 1 << 17) -> np.ndarray:
    """y = A_bc x (bc=True) or y = A x, cell by cell, without forming A.

    Same definition as the assembled operator; element matrices are formed in
    chunks and the local products scattered with np.bincount.
    """
    x = np.asarray(x, dtype=np.float64)
    xin = x.copy()
    if bc:
        xin[level.boundary] = 0.0
    y = np.zeros(level.n_dofs)
    C = level.n_cells
    for s in range(0, C, chunk):
        sl = slice(s, min(C, s + chunk))
        Ae = element_matrices(level, k_vertex, sl)
        dofs = level.cell_dofs[sl]
        yk = np.einsum("cij,cj->ci", Ae, xin[dofs])
        y += np.bincount(dofs.ravel(), weights=yk.ravel(), minlength=level.n_dofs)
    if bc:
        y[level.boundary] = x[level.boundary]
    return y


def action_at(n: int, p: int, vert_xyz: np.ndarray, x: np.ndarray, sample: np.ndarray,
              k_vertex: np.ndarray | None = None, bc: bool = True) -> np.ndarray:
    """(A_bc x)_i (bc=True) or (A x)_i for the sampled dofs i only, on the P_p space of the
    n^3 x 6 mesh with vertex positions vert_xyz (((n+1)^3, 3)).

    The same definition as matfree_action, summed over the cells around each sampled dof
    instead of all cells: row i of A x is the sum over the cells whose closure holds dof i of
    their local products, and those cells lie in the cubes whose p-lattice box contains the
    dof's lattice point.  Those cubes' six tetrahedra are formed (a superset; the other cells'
    rows do not include dof i), their element matrices built from the same reference tensors,
    and the local products summed into the sampled rows.  Used for checks at sizes where the
    full action is too slow to compute.
    """
    from .mesh import cube_cells, vertex_id
    sample = np.asarray(sample, dtype=np.int64)
    L = p * n + 1
    ijk = np.stack([sample % L, (sample // L) % L, sample // (L * L)], axis=1)
    cand = []
    for d in range(3):
        lo = np.clip((ijk[:, d] - 1) // p, 0, n - 1)
        hi = np.clip(ijk[:, d] // p, 0, n - 1)
        cand.append((lo, hi))
    corners = []
    for bits in range(8):
        c = np.stack([cand[d][(bits >> d) & 1] for d in range(3)], axis=1)
        corners.append(c)
    corners = np.unique(np.concatenate(corners), axis=0)
    cells_ijk = cube_cells(corners)
    cell_vert = vertex_id(n, cells_ijk)
    mi = np.array(refelem.node_multi_indices(p), dtype=np.int64)
    lat = np.einsum("li,cid->cld", mi, cells_ijk)
    cell_dofs = lat[..., 0] + L * (lat[..., 1] + L * lat[..., 2])
    xyz = vert_xyz[cell_vert]
    J = np.stack([xyz[:, 1] - xyz[:, 0], xyz[:, 2] - xyz[:, 0], xyz[:, 3] - xyz[:, 0]], axis=2)
    det = np.linalg.det(J)
    Jinv = np.linalg.inv(J)
    G = np.abs(det)[:, None, None] * np.einsum("cai,cbi->cab", Jinv, Jinv)
    if k_vertex is None:
        Ae = np.einsum("cab,abij->cij", G, refelem.S(p))
    else:
        kc = np.asarray(k_vertex, dtype=np.float64)[cell_vert]
        Ae = np.einsum("cv,cab,vabij->cij", kc, G, refelem.T(p))
    xl = np.asarray(x, dtype=np.float64)[cell_dofs]
    if bc:
        on_bnd = np.any((lat == 0) | (lat == p * n), axis=2)
        xl = np.where(on_bnd, 0.0, xl)
    yk = np.einsum("cij,cj->ci", Ae, xl)
    uniq, inv = np.unique(sample, return_inverse=True)
    flat = cell_dofs.ravel()
    pos = np.searchsorted(uniq, flat)
    hit = (pos < uniq.size) & (uniq[np.minimum(pos, uniq.size - 1)] == flat)
    acc = np.zeros(uniq.size)
    np.add.at(acc, pos[hit], yk.ravel()[hit])
    y = acc[inv]
    if bc:
        s_bnd = np.any((ijk == 0) | (ijk == p * n), axis=1)
        y[s_bnd] = np.asarray(x, dtype=np.float64)[sample[s_bnd]]
    return y


def diagonal(A: sp.csr_matrix) -> np.ndarray:
    return A.diagonal().copy()


def load_vector(level: Level, f, degree: int) -> np.ndarray:
    """b_i = int f phi_i by a conical-product rule of the given degree."""
    from .quadrature import conical_product_rule
    pts, wts = conical_product_rule(degree)
    phi = refelem.eval_basis(level.p, pts)                  # (nq, nloc)
    x = level.cell_xyz()                                     # (C, 4, 3)
    J = np.stack([x[:, 1] - x[:, 0], x[:, 2] - x[:, 0], x[:, 3] - x[:, 0]], axis=2)
    det = np.abs(np.linalg.det(J))
    phys = x[:, 0][:, None, :] + np.einsum("cdk,qk->cqd", J, pts)  # (C, nq, 3)
    fq = f(phys.reshape(-1, 3)).reshape(phys.shape[:2])
    be = np.einsum("c,q,cq,qi->ci", det, wts, fq, phi)
    return np.bincount(level.cell_dofs.ravel(), weights=be.ravel(), minlength=level.n_dofs)


def l2_error(level: Level, uh: np.ndarray, u_exact, degree: int) -> float:
    """||u_h - u||_{L2} cell by cell with a conical-product rule."""
    from .quadrature import conical_product_rule
    pts, wts = conical_product_rule(degree)
    phi = refelem.eval_basis(level.p, pts)
    x = level.cell_xyz()
    J = np.stack([x[:, 1] - x[:, 0], x[:, 2] - x[:, 0], x[:, 3] - x[:, 0]], axis=2)
    det = np.abs(np.linalg.det(J))
    phys = x[:, 0][:, None, :] + np.einsum("cdk,qk->cqd", J, pts)
    ue = u_exact(phys.reshape(-1, 3)).reshape(phys.shape[:2])
    uq = np.einsum("qi,ci->cq", phi, uh[level.cell_dofs])
    return float(np.sqrt(np.einsum("c,q,cq->", det, wts, (uq - ue) ** 2)))
