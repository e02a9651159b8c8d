"""Pins for the oracle's additive vertex-star patch preconditioner (Listing 2's
star patches around vertices), checked against facts fixed by the mesh and
the mathematics rather than against the oracle's own formulas:

* P1: a vertex star carries only the vertex's own dof, so the preconditioner
  is point Jacobi, z = r / diag(A_bc).
* Star sizes of a vertex whose star is interior: its link in the six-tetrahedra
  split is a triangulated sphere with 14 vertices, 36 edges and 24 triangles
  (Euler characteristic 2), so a P_p star holds
  1 + (p-1) 14 + C(p-1, 2) 36 + C(p-1, 3) 24 dofs: 1, 15, 65 for p = 1, 2, 3.
* With A = I every interior dof is counted once per vertex of the entity that
  carries it (1 for a vertex, 2 for an edge, 3 for a face, 4 for a cell),
  boundary dofs pass through.
* A_v equals the sum over the cells around v of their element matrices
  restricted to the star nodes (every cell coupling two star dofs contains v).
* The preconditioner is symmetric positive definite.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import fem_inputs
from oracle import assemble, patch, refelem
from oracle import mesh as om


def _level(n, p, jitter=0.0, seed=6):
    jit = fem_inputs.jitter_offsets(n, jitter, seed=seed) if jitter else None
    return om.single_level(n, p, jit)


def _abc(level, k=None):
    return assemble.apply_bc(assemble.stiffness(level, k), level.boundary)


def test_p1_star_patch_is_point_jacobi():
    lv = _level(4, 1, jitter=0.15)
    k = fem_inputs.k_exp_fourier(lv.vert_xyz, seed=1)
    A = _abc(lv, k)
    pts = patch.star_patches(lv)
    assert all(idx.size <= 1 for idx in pts)
    r = fem_inputs.uniform_vector(lv.n_dofs, seed=0)
    z = patch.apply_patch_pc(pts, patch.patch_inverses(A, pts), lv.boundary, r)
    np.testing.assert_allclose(z, r / A.diagonal(), rtol=1e-13, atol=0)


@pytest.mark.parametrize("p,size", [(1, 1), (2, 15), (3, 65)])
def test_interior_star_size_from_vertex_link(p, size):
    V, E, F, T = 14, 36, 24, 24
    assert V - E + F == 2
    assert size == 1 + (p - 1) * V + (p - 1) * (p - 2) // 2 * E + (p - 1) * (p - 2) * (p - 3) // 6 * T
    n = 3
    lv = _level(n, p)
    pts = patch.star_patches(lv)
    for ijk in [(1, 1, 1), (1, 2, 1), (2, 2, 2)]:
        v = int(om.vertex_id(n, np.array(ijk)))
        assert pts[v].size == size
    # boundary vertices keep a (smaller) patch of interior dofs, never a boundary dof
    for v in range(lv.n_vertices):
        assert not lv.boundary[pts[v]].any()


@pytest.mark.parametrize("p", [1, 2, 3])
def test_identity_matrix_counts_entity_vertices(p):
    lv = _level(3, p)
    pts = patch.star_patches(lv)
    N = lv.n_dofs
    inv = patch.patch_inverses(sp.identity(N, format="csr"), pts)
    r = fem_inputs.uniform_vector(N, seed=0)
    z = patch.apply_patch_pc(pts, inv, lv.boundary, r)
    # number of vertices of the entity carrying each dof: nonzero entries of its multi-index
    mi = np.array(refelem.node_multi_indices(p))
    count = np.zeros(N, dtype=np.int64)
    count[lv.cell_dofs.ravel()] = np.tile((mi > 0).sum(axis=1), lv.n_cells)
    want = np.where(lv.boundary, r, count * r)
    np.testing.assert_allclose(z, want, rtol=1e-15, atol=0)
    if p == 2:
        assert set(np.unique(count[~lv.boundary])) == {1, 2}


@pytest.mark.parametrize("p", [2, 3])
def test_patch_matrix_is_sum_of_star_element_matrices(p):
    lv = _level(2, p, jitter=0.2)
    k = fem_inputs.k_exp_fourier(lv.vert_xyz, seed=1)
    A = _abc(lv, k)
    pts = patch.star_patches(lv)
    Ae = assemble.element_matrices(lv, k)
    mi = np.array(refelem.node_multi_indices(p))
    for v in range(lv.n_vertices):
        idx = pts[v]
        if idx.size == 0:
            continue
        pos = {int(d): a for a, d in enumerate(idx)}
        Av = np.zeros((idx.size, idx.size))
        for c in range(lv.n_cells):
            loc = np.nonzero(lv.cell_vert[c] == v)[0]
            if loc.size == 0:
                continue
            nodes = [a for a in range(mi.shape[0]) if mi[a, loc[0]] > 0 and int(lv.cell_dofs[c, a]) in pos]
            for a in nodes:
                for b in nodes:
                    Av[pos[int(lv.cell_dofs[c, a])], pos[int(lv.cell_dofs[c, b])]] += Ae[c, a, b]
        np.testing.assert_allclose(Av, A[idx][:, idx].toarray(), rtol=1e-12, atol=1e-14)


def test_single_interior_dof_covered_twice():
    # Kuhn(1), P2: the only interior dof is the midpoint of the main diagonal, whose two end
    # vertices each carry it in their star
    lv = _level(1, 2)
    A = _abc(lv)
    pts = patch.star_patches(lv)
    g = int(np.nonzero(~lv.boundary)[0][0])
    r = fem_inputs.uniform_vector(lv.n_dofs, seed=2)
    z = patch.apply_patch_pc(pts, patch.patch_inverses(A, pts), lv.boundary, r)
    assert z[g] == pytest.approx(2.0 * r[g] / A[g, g], rel=1e-14)
    assert sum(int(idx.size) for idx in pts) == 2


def test_preconditioner_symmetric_positive_definite():
    lv = _level(2, 2, jitter=0.1)
    k = fem_inputs.k_exp_fourier(lv.vert_xyz, seed=1)
    A = _abc(lv, k)
    pts = patch.star_patches(lv)
    inv = patch.patch_inverses(A, pts)
    N = lv.n_dofs
    P = np.stack([patch.apply_patch_pc(pts, inv, lv.boundary, e) for e in np.eye(N)], axis=1)
    np.testing.assert_allclose(P, P.T, rtol=0, atol=1e-12 * np.abs(P).max())
    assert np.linalg.eigvalsh(0.5 * (P + P.T)).min() > 0


def test_cg_lanczos_reaches_largest_eigenvalue():
    # with as many CG steps as needed the CG-Lanczos estimate is the largest eigenvalue of B A,
    # computed here by a dense eigen-solver (patches) and checked for B = D^-1 as well
    from oracle import solvers
    lv = _level(2, 2, jitter=0.1)
    k = fem_inputs.k_exp_fourier(lv.vert_xyz, seed=1)
    A = _abc(lv, k)
    pts = patch.star_patches(lv)
    inv = patch.patch_inverses(A, pts)
    N = lv.n_dofs
    prec = lambda v: patch.apply_patch_pc(pts, inv, lv.boundary, v)
    Bd = np.stack([prec(e) for e in np.eye(N)], axis=1)
    lam = np.max(np.linalg.eigvals(Bd @ A.toarray()).real)
    assert solvers.pcg_lanczos_lmax(A, prec, steps=80) == pytest.approx(lam, rel=1e-9)
    dinv = 1.0 / A.diagonal()
    lam_j = np.max(np.linalg.eigvals(dinv[:, None] * A.toarray()).real)
    assert solvers.pcg_lanczos_lmax(A, lambda v: dinv * v, steps=80) == pytest.approx(lam_j, rel=1e-9)
    # a few steps underestimate, never overestimate (Ritz values lie inside the spectrum)
    assert solvers.pcg_lanczos_lmax(A, prec, steps=10) <= lam * (1 + 1e-12)


def test_patch_smoothed_vcycle_contracts():
    # two-level cycle with the patch-preconditioned Chebyshev smoother: the error propagation
    # I - B_mg A has A-norm below 1 (a convergent multigrid iteration)
    from oracle import solvers
    levels = om.hierarchy(2, 1, 2, fem_inputs.jitter_offsets(2, 0.1))
    mg = solvers.MGHierarchy(levels, None, smoother="patch")
    A = mg.levels[-1].A.toarray()
    N = A.shape[0]
    E = np.eye(N) - np.stack([mg.vcycle(A[:, j]) for j in range(N)], axis=1)
    Ls = np.linalg.cholesky(A)
    rho = np.linalg.norm(Ls.T @ E @ np.linalg.inv(Ls.T), 2)
    assert rho < 0.5


@pytest.mark.parametrize("n,p,jit", [(3, 2, 0.15), (2, 3, 0.1)])
def test_pointwise_patch_values_match_global_definition(n, p, jit):
    # the one-dof-at-a-time evaluation used at large sizes equals the global construction
    lv = _level(n, p, jitter=jit)
    k = fem_inputs.k_exp_fourier(lv.vert_xyz, seed=1)
    A = _abc(lv, k)
    pts = patch.star_patches(lv)
    r = fem_inputs.uniform_vector(lv.n_dofs, seed=0)
    z = patch.apply_patch_pc(pts, patch.patch_inverses(A, pts), lv.boundary, r)
    sample = np.arange(lv.n_dofs)
    np.testing.assert_allclose(patch.patch_pc_at(lv, k, r, sample), z, rtol=1e-12, atol=1e-14 * np.abs(z).max())
