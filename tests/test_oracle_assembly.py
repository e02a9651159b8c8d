"""Pins for the oracle's assembled operators.

* P1 on the six-tetrahedra split is h times the 7-point finite-difference
  Laplacian (diagonal 6h, axis neighbours -h, every other coupling zero).
* A . 1 = 0 without boundary conditions.
* Exact reproduction: for ell linear, (A ell)_i = 0 on interior rows; for q
  quadratic (p >= 2), (A q)_i = -lap(q) int phi_i; for c cubic (p = 3),
  (A c)_i = (M (-lap c))_i, since -lap(c) is linear and in the space.
* Exact reproduction with a coefficient: for k = ell linear (its P1
  interpolant is exact) and q of degree p, the interior rows of A(k) q equal
  (M f)_i with f = -grad(ell).grad(q) - ell lap(q) of degree p - 1.  This pins
  the P1-coefficient tensor T^{v,ab}: permuting its vertex weights fails it.
* Structure: nnz counts from the sparsity pattern.
"""
import numpy as np
import pytest

import fem_inputs
from oracle import assemble
from oracle import mesh as om


def _lap7(n):
    """h * 7-point Laplacian with Dirichlet identity rows on the (n+1)^3 lattice."""
    h = 1.0 / n
    L = n + 1
    N = L ** 3
    A = np.zeros((N, N))
    for k in range(L):
        for j in range(L):
            for i in range(L):
                r = i + L * (j + L * k)
                if min(i, j, k) == 0 or max(i, j, k) == n:
                    A[r, r] = 1.0
                    continue
                A[r, r] = 6 * h
                for d in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                    ii, jj, kk = i + d[0], j + d[1], k + d[2]
                    if min(ii, jj, kk) == 0 or max(ii, jj, kk) == n:
                        continue
                    A[r, ii + L * (jj + L * kk)] = -h
    return A


@pytest.mark.parametrize("n", [2, 4])
def test_p1_is_7point(n):
    lev = om.single_level(n, 1)
    A = assemble.apply_bc(assemble.stiffness(lev), lev.boundary).toarray()
    assert np.max(np.abs(A - _lap7(n))) < 1e-14


@pytest.mark.parametrize("p,coef", [(1, 15), (2, 230), (3, 1311)])
def test_nnz_structure(p, coef):
    poly = {1: (15, 21, 9, 1), 2: (230, 138, 24, 1), 3: (1311, 459, 45, 1)}[p]
    for n in (1, 2, 3):
        A = assemble.stiffness(om.single_level(n, p))
        A.eliminate_zeros()
        pattern_nnz = np.unique(np.stack([np.repeat(om.single_level(n, p).cell_dofs, refelem_n(p), axis=1).ravel(),
                                          np.tile(om.single_level(n, p).cell_dofs, (1, refelem_n(p))).ravel()]),
                                axis=1).shape[1]
        assert pattern_nnz == poly[0] * n ** 3 + poly[1] * n ** 2 + poly[2] * n + poly[3]


def refelem_n(p):
    return (p + 1) * (p + 2) * (p + 3) // 6


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("jit", [False, True])
@pytest.mark.parametrize("kvar", [False, True])
def test_constants_in_kernel_and_symmetry(p, jit, kvar):
    n = 3
    lev = om.single_level(n, p, fem_inputs.jitter_offsets(n, 0.15) if jit else None)
    k = fem_inputs.k_exp_fourier(lev.vert_xyz) if kvar else None
    A = assemble.stiffness(lev, k)
    scale = abs(A).max()
    assert np.max(np.abs(A @ np.ones(lev.n_dofs))) < 1e-13 * scale
    assert abs(A - A.T).max() < 1e-14 * scale


def _interior_rows(lev):
    return lev.interior()


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("jit", [False, True])
def test_linear_exactness(p, jit):
    n = 3
    lev = om.single_level(n, p, fem_inputs.jitter_offsets(n, 0.15) if jit else None)
    A = assemble.stiffness(lev)
    xyz = lev.dof_xyz()
    ell = 0.3 + 1.1 * xyz[:, 0] - 0.7 * xyz[:, 1] + 2.3 * xyz[:, 2]
    r = (A @ ell)[_interior_rows(lev)]
    assert np.max(np.abs(r)) < 1e-13


@pytest.mark.parametrize("p", [2, 3])
@pytest.mark.parametrize("jit", [False, True])
def test_quadratic_exactness(p, jit):
    from oracle import refelem
    n = 3
    lev = om.single_level(n, p, fem_inputs.jitter_offsets(n, 0.15) if jit else None)
    A = assemble.stiffness(lev)
    x, y, z = lev.dof_xyz().T
    q = 1.0 + x * x - 2.0 * y * y + 3.0 * z * z + 0.5 * x * y - z * x + 0.25 * y * z + x
    minus_lap_q = -(2.0 - 4.0 + 6.0)
    # int phi_i over the mesh, by assembling the reference integrals
    _, det = lev.geometric_factors()
    wi = np.bincount(lev.cell_dofs.ravel(),
                     weights=(det[:, None] * refelem.basis_integrals(p)[None, :]).ravel(),
                     minlength=lev.n_dofs)
    I = _interior_rows(lev)
    assert np.max(np.abs((A @ q)[I] - minus_lap_q * wi[I])) < 1e-13


@pytest.mark.parametrize("jit", [False, True])
def test_cubic_exactness_p3(jit):
    n = 3
    lev = om.single_level(n, 3, fem_inputs.jitter_offsets(n, 0.15) if jit else None)
    A = assemble.stiffness(lev)
    M = assemble.mass(lev)
    x, y, z = lev.dof_xyz().T
    c = x ** 3 + 2 * y ** 2 * z - x * y * z + 0.5 * z ** 3 + y
    minus_lap_c = -(6 * x + 4 * z + 3 * z)
    I = _interior_rows(lev)
    assert np.max(np.abs((A @ c)[I] - (M @ minus_lap_c)[I])) < 1e-13


@pytest.mark.parametrize("p", [1, 2, 3])
def test_mass_total(p):
    lev = om.single_level(3, p, fem_inputs.jitter_offsets(3, 0.15))
    M = assemble.mass(lev)
    assert abs(M.sum() - 1.0) < 1e-13


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("kvar", [False, True])
def test_matfree_matches_csr(p, kvar):
    n = 3
    lev = om.single_level(n, p, fem_inputs.jitter_offsets(n, 0.15))
    k = fem_inputs.k_exp_fourier(lev.vert_xyz) if kvar else None
    x = fem_inputs.uniform_vector(lev.n_dofs, 0)
    A = assemble.apply_bc(assemble.stiffness(lev, k), lev.boundary)
    y1 = A @ x
    y2 = assemble.matfree_action(lev, x, k, bc=True, chunk=37)
    assert np.linalg.norm(y1 - y2) <= 1e-14 * np.linalg.norm(y1)
    y3 = assemble.matfree_action(lev, x, k, bc=False)
    assert np.linalg.norm(assemble.stiffness(lev, k) @ x - y3) <= 1e-14 * np.linalg.norm(y3)


def test_kvar_constant_equals_scaled():
    lev = om.single_level(2, 3)
    k = np.full(lev.n_vertices, 2.5)
    A1 = assemble.stiffness(lev, k)
    A0 = assemble.stiffness(lev)
    assert abs(A1 - 2.5 * A0).max() < 1e-14


def _var_k_exactness_residual(p, jit, T_override=None, monkeypatch=None):
    """Interior rows of A(k) q - M f for k = ell (linear, so its P1 interpolant is exact), q a
    polynomial of degree p and f = -div(ell grad q) = -grad(ell).grad(q) - ell lap(q), which has
    degree p - 1 and so lies in the space: a(q, phi_i) = int f phi_i = (M f)_i exactly for every
    interior test function (weak form of Section 2 eq. (4) with a coefficient)."""
    from oracle import refelem
    if T_override is not None:
        monkeypatch.setattr(refelem, "T", T_override)
    n = 3
    lev = om.single_level(n, p, fem_inputs.jitter_offsets(n, 0.15) if jit else None)
    gl = np.array([0.8, -0.6, 1.3])                      # grad(ell)
    vx = lev.vert_xyz
    k = 2.0 + vx @ gl                                    # ell > 0 on the unit cube
    x, y, z = lev.dof_xyz().T
    if p == 1:
        q = 0.4 + 1.5 * x - 0.9 * y + 0.7 * z
        gq = np.stack([np.full_like(x, 1.5), np.full_like(x, -0.9), np.full_like(x, 0.7)])
        lap_q = np.zeros_like(x)
    elif p == 2:
        q = 1.0 + x * x - 2.0 * y * y + 3.0 * z * z + 0.5 * x * y - z * x + 0.25 * y * z + x
        gq = np.stack([2 * x + 0.5 * y - z + 1.0, -4 * y + 0.5 * x + 0.25 * z, 6 * z - x + 0.25 * y])
        lap_q = np.full_like(x, 2.0 - 4.0 + 6.0)
    else:
        q = x ** 3 + 2 * y ** 2 * z - x * y * z + 0.5 * z ** 3 + y + x * z
        gq = np.stack([3 * x ** 2 - y * z + z, 4 * y * z - x * z + 1.0, 2 * y ** 2 - x * y + 1.5 * z ** 2 + x])
        lap_q = 6 * x + 4 * z + 3 * z
    ell = 2.0 + np.stack([x, y, z]).T @ gl
    f = -(gl @ gq) - ell * lap_q
    A = assemble.stiffness(lev, k)
    M = assemble.mass(lev)
    I = _interior_rows(lev)
    return np.max(np.abs((A @ q)[I] - (M @ f)[I])), np.max(np.abs(M @ f))


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("jit", [False, True])
def test_variable_coefficient_exactness(p, jit):
    err, scale = _var_k_exactness_residual(p, jit)
    assert err < 1e-13 * max(1.0, scale)


@pytest.mark.parametrize("p", [2, 3])
def test_variable_coefficient_exactness_catches_vertex_permutation(p, monkeypatch):
    """The exactness pin above fails when the barycentric weights l_v of the P1-coefficient
    tensor T^{v,ab} are permuted among the vertices (a mistake that A.1 = 0, symmetry, the
    adjoint identity and finite differences all accept)."""
    from oracle import refelem
    T0 = refelem.T(p)
    for perm in ((1, 0, 2, 3), (3, 1, 2, 0), (0, 2, 3, 1)):
        err, scale = _var_k_exactness_residual(p, True, T_override=lambda _p, P=perm: T0[list(P)],
                                               monkeypatch=monkeypatch)
        assert err > 1e-4 * scale, perm


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("kvar", [False, True])
@pytest.mark.parametrize("bc", [True, False])
def test_action_at_sampled_rows_equals_full_action(p, kvar, bc):
    """The sampled-row evaluation (cells around each sampled dof only) equals the full action on
    every dof of small jittered meshes, boundary rows included, with repeated sample entries."""
    n = 3
    lev = om.single_level(n, p, fem_inputs.jitter_offsets(n, 0.15))
    k = fem_inputs.k_exp_fourier(lev.vert_xyz) if kvar else None
    x = fem_inputs.uniform_vector(lev.n_dofs, 0)
    y = assemble.matfree_action(lev, x, k, bc=bc)
    every = np.arange(lev.n_dofs)
    ys = assemble.action_at(n, p, lev.vert_xyz, x, every, k, bc=bc)
    assert np.max(np.abs(ys - y)) <= 1e-14 * np.max(np.abs(y))
    sub = np.array([5, 0, lev.n_dofs - 1, 5, 17])
    ysub = assemble.action_at(n, p, lev.vert_xyz, x, sub, k, bc=bc)
    assert np.max(np.abs(ysub - y[sub])) <= 1e-14 * np.max(np.abs(y))
