"""Prolongation between nested P_p spaces, by evaluating coarse basis functions
at fine nodes (Section 4: the coarse correction is transferred to the finer
mesh; uniform refinement makes the spaces nested, so prolongation is exact
interpolation and restriction is its transpose).

Construction (deliberately point-by-point): every fine dof sits at a fine
lattice point; in coarse-lattice units that point lies in some coarse cube,
and inside the cube in the tetrahedron whose axis order sorts the fractional
coordinates decreasingly.  Its barycentric coordinates in that tetrahedron
are read off the sorted fractions, and the coarse basis functions of that
cell are evaluated there.

Parity: reproduction of coarse polynomials of degree <= p and the Galerkin
identity P^T A_f P = A_c are pinned in tests/test_oracle_solvers.py.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import refelem
from .mesh import Level, dof_lattice


def _locate(n_c: int, pts: np.ndarray):
    """pts in coarse-cube units (float, in [0, n_c]^3).  Returns the cube
    corner (N,3), the permutation index order (N,3) and barycentric coords (N,4)
    of the containing Kuhn tetrahedron."""
    cube = np.minimum(np.floor(pts).astype(np.int64), n_c - 1)
    f = pts - cube                                       # fractions in [0, 1]
    order = np.argsort(-f, axis=1, kind="stable")        # axes by decreasing fraction
    fs = np.take_along_axis(f, order, axis=1)            # f_s0 >= f_s1 >= f_s2
    lam = np.stack([1.0 - fs[:, 0], fs[:, 0] - fs[:, 1], fs[:, 1] - fs[:, 2], fs[:, 2]], axis=1)
    return cube, order, lam


def prolongation(coarse: Level, fine: Level) -> sp.csr_matrix:
    """P (n_fine x n_coarse): P[i, j] = phi^c_j(x_i)."""
    assert fine.n == 2 * coarse.n and fine.p == coarse.p
    p = coarse.p
    n_c = coarse.n
    Lc = p * n_c + 1
    latt = dof_lattice(fine.n, p).astype(np.float64)      # fine lattice, spacing h_f / p
    pts = latt / (2 * p)                                   # coarse-cube units
    cube, order, lam = _locate(n_c, pts)
    # coarse cell's vertex integer coordinates along the path
    V = np.zeros((pts.shape[0], 4, 3), dtype=np.int64)
    V[:, 0] = cube
    for s in range(3):
        V[:, s + 1] = V[:, s]
        np.add.at(V[:, s + 1], (np.arange(pts.shape[0]), order[:, s]), 1)
    # barycentric -> reference coordinates (l1, l2, l3)
    vals = refelem.eval_basis(p, lam[:, 1:])               # (Nf, nloc)
    mi = np.array(refelem.node_multi_indices(p), dtype=np.int64)
    lat_c = np.einsum("li,nid->nld", mi, V)                # coarse lattice coords of cell nodes
    cdofs = lat_c[..., 0] + Lc * (lat_c[..., 1] + Lc * lat_c[..., 2])
    rows = np.repeat(np.arange(pts.shape[0]), mi.shape[0])
    P = sp.coo_matrix((vals.ravel(), (rows, cdofs.ravel())), shape=(fine.n_dofs, coarse.n_dofs)).tocsr()
    P.data[np.abs(P.data) < 1e-14] = 0.0
    P.eliminate_zeros()
    return P
