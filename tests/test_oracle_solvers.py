"""Pins for the oracle's solvers, multigrid pieces and manufactured solutions.

* CG against a dense LAPACK solve on tiny problems (brute force).
* Jacobi-CG on P1: the operator is h times the 7-point Laplacian, with
  condition number cot^2(pi / 2n); CG needs at most about 60 iterations for
  1e-10 at n = 8.
* O(h^{p+1}) L2 convergence for the sine manufactured solution and for the
  paper's manufactured solution (Section 2, eqs. 2-3 with a = 1, b = 2).
* Chebyshev damping on P1 sine modes equals T_2((theta - mu)/delta) /
  T_2(theta/delta) exactly (the modes are eigenvectors of D^-1 A).
* V-cycle symmetry, Galerkin identity, polynomial reproduction by P.
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import fem_inputs
from oracle import assemble, solvers, transfer
from oracle import mesh as om


def _system(n, p, jit=False, kvar=False):
    lev = om.single_level(n, p, fem_inputs.jitter_offsets(n, 0.15) if jit else None)
    k = fem_inputs.k_exp_fourier(lev.vert_xyz) if kvar else None
    A = assemble.apply_bc(assemble.stiffness(lev, k), lev.boundary)
    return lev, A


@pytest.mark.parametrize("n,p", [(2, 1), (2, 2), (2, 3), (3, 2)])
def test_cg_matches_dense_solve(n, p):
    lev, A = _system(n, p, jit=True, kvar=True)
    b = assemble.mass(lev) @ fem_inputs.sin3_f(lev.dof_xyz())
    b[lev.boundary] = 0
    x_dense = np.linalg.solve(A.toarray(), b)
    x, it, _ = solvers.cg(A, b, rtol=1e-13)
    assert np.linalg.norm(x - x_dense) <= 1e-11 * np.linalg.norm(x_dense)
    assert np.linalg.norm(solvers.direct_solve(A, b) - x_dense) <= 1e-12 * np.linalg.norm(x_dense)


def test_jacobi_cg_iteration_bound_p1_n8():
    lev, A = _system(8, 1)
    b = assemble.load_vector(lev, fem_inputs.sin3_f, 6)
    b[lev.boundary] = 0
    dinv = 1.0 / A.diagonal()
    x, it, hist = solvers.cg(A, b, rtol=1e-10, M=lambda r: dinv * r)
    kappa = 1.0 / math.tan(math.pi / 16) ** 2
    bound = math.ceil(0.5 * math.sqrt(kappa) * math.log(2.0 / 1e-10))
    assert it <= bound <= 60
    assert np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b)


def _mms_errors(p, ns, u, f):
    errs = []
    for n in ns:
        lev, A = _system(n, p)
        b = assemble.load_vector(lev, f, 2 * p + 4)
        b[lev.boundary] = 0
        uh = solvers.direct_solve(A, b)
        errs.append(assemble.l2_error(lev, uh, u, 2 * p + 4))
    return np.array(errs)


@pytest.mark.parametrize("p,ns", [(1, (4, 8, 16)), (2, (4, 8, 16)), (3, (2, 4, 8))])
def test_mms_rates_sin3(p, ns):
    e = _mms_errors(p, ns, fem_inputs.sin3_u, fem_inputs.sin3_f)
    rates = np.log2(e[:-1] / e[1:])
    assert rates[-1] >= p + 1 - 0.15, rates


@pytest.mark.parametrize("p,ns", [(2, (4, 8, 16)), (3, (4, 6, 8))])
def test_mms_rates_paper_solution(p, ns):
    e = _mms_errors(p, ns, fem_inputs.paper_u, fem_inputs.paper_f)
    rates = np.log(e[:-1] / e[1:]) / np.log(np.array(ns[1:]) / np.array(ns[:-1]))
    assert rates[-1] >= p + 1 - 0.2, rates


def test_paper_f_is_minus_laplacian_of_paper_u():
    # eqs. 2 and 3 agree: -lap(u) = f, checked with a 4th-order central difference
    rng = np.random.default_rng(11)
    pts = rng.uniform(0.1, 0.9, (50, 3))
    h = 1e-3
    lap = np.zeros(len(pts))
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        lap += (-fem_inputs.paper_u(pts + 2 * e) + 16 * fem_inputs.paper_u(pts + e)
                - 30 * fem_inputs.paper_u(pts) + 16 * fem_inputs.paper_u(pts - e)
                - fem_inputs.paper_u(pts - 2 * e)) / (12 * h * h)
    f = fem_inputs.paper_f(pts)
    assert np.max(np.abs(-lap - f)) < 1e-5 * np.max(np.abs(f))


def test_sin3_energy_and_norm():
    # u_h^T A u_h -> int |grad u|^2 = 3 pi^2 / 8 and ||u||^2 = 1/8 for the sine solution
    lev, A = _system(8, 3)
    b = assemble.load_vector(lev, fem_inputs.sin3_f, 10)
    b[lev.boundary] = 0
    uh = solvers.direct_solve(A, b)
    assert abs(uh @ (A @ uh) - 3 * math.pi ** 2 / 8) < 1e-5
    M = assemble.mass(lev)
    assert abs(uh @ (M @ uh) - 1 / 8) < 2e-6


def test_chebyshev_damping_closed_form():
    n = 8
    lev, A = _system(n, 1)
    dinv = 1.0 / A.diagonal()
    lmax = (2.0 / 3.0) * 3 * math.sin((n - 1) * math.pi / (2 * n)) ** 2
    lo, hi = 0.1, 1.1
    theta = 0.5 * (hi + lo) * lmax
    delta = 0.5 * (hi - lo) * lmax
    T2 = lambda t: 2 * t * t - 1
    ijk = om.dof_lattice(n, 1)
    for m in [(1, 1, 1), (3, 5, 2), (7, 7, 7), (4, 1, 6)]:
        v = np.prod(np.sin(np.pi * np.array(m)[None, :] * ijk / n), axis=1)
        v[lev.boundary] = 0
        mu = (2.0 / 3.0) * sum(math.sin(mi * math.pi / (2 * n)) ** 2 for mi in m)
        out = solvers.chebyshev_smooth(A, dinv, np.zeros(lev.n_dofs), v, lmax, 2, lo, hi)
        factor = T2((theta - mu) / delta) / T2(theta / delta)
        assert np.max(np.abs(out - factor * v)) < 1e-13


def test_lanczos_estimate_bounds():
    n = 8
    _, A = _system(n, 1)
    dinv = 1.0 / A.diagonal()
    true = (2.0 / 3.0) * 3 * math.sin((n - 1) * math.pi / (2 * n)) ** 2
    est = solvers.lanczos_lmax(A, dinv, 10)
    assert 0.85 * true <= est <= true * (1 + 1e-12)


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("jit", [False, True])
def test_prolongation_reproduces_polynomials(p, jit):
    coarse, fine = om.hierarchy(2, 1, p, fem_inputs.jitter_offsets(2, 0.15) if jit else None)
    P = transfer.prolongation(coarse, fine)
    for f in (lambda x: 1.0 + 0 * x[:, 0],
              lambda x: x[:, 0] - 2 * x[:, 1] + 0.5 * x[:, 2],
              lambda x: x[:, 0] ** p + x[:, 1] ** (p - 1) * x[:, 2] - x[:, 2] ** p):
        uc = f(coarse.dof_xyz())
        uf = f(fine.dof_xyz())
        assert np.max(np.abs(P @ uc - uf)) < 1e-13
    # rows of P sum to one (constants are reproduced) and P is exact at coarse nodes
    assert np.allclose(np.asarray(P.sum(axis=1)).ravel(), 1.0, atol=1e-14)


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("jit", [False, True])
def test_galerkin_identity(p, jit):
    coarse, fine = om.hierarchy(2, 1, p, fem_inputs.jitter_offsets(2, 0.15) if jit else None)
    P = transfer.prolongation(coarse, fine)
    Af = assemble.stiffness(fine)
    Ac = assemble.stiffness(coarse)
    diff = abs(P.T @ Af @ P - Ac).max()
    assert diff < 1e-13 * abs(Ac).max()


@pytest.mark.parametrize("p", [1, 2])
def test_vcycle_symmetric_and_mgcg_converges(p):
    levels = om.hierarchy(2, 2, p, fem_inputs.jitter_offsets(2, 0.1))
    k = fem_inputs.k_exp_fourier(levels[-1].vert_xyz)
    mg = solvers.MGHierarchy(levels, k)
    nf = levels[-1].n_dofs
    rng = np.random.default_rng(0)
    x = rng.standard_normal(nf)
    y = rng.standard_normal(nf)
    x[levels[-1].boundary] = 0
    y[levels[-1].boundary] = 0
    bx, by = mg.vcycle(x), mg.vcycle(y)
    assert abs(bx @ y - x @ by) <= 1e-12 * abs(bx @ y)
    assert bx @ x > 0
    b = assemble.mass(levels[-1]) @ fem_inputs.sin3_f(levels[-1].dof_xyz())
    b[levels[-1].boundary] = 0
    u, it, hist = mg.solve(b, rtol=1e-10)
    A = mg.levels[-1].A
    u_ref = spla.spsolve(A.tocsc(), b)
    assert np.linalg.norm(u - u_ref) <= 1e-8 * np.linalg.norm(u_ref)
    assert it <= 20


@pytest.mark.parametrize("p,n0,refine", [(1, 2, 3), (2, 2, 2)])
def test_fmg_reaches_discretisation_accuracy(p, n0, refine):
    """One full-multigrid cycle (Listing 2's solver) lands within a small factor of the exact
    discrete solution's L2 error for the sine solution (the textbook FMG property: the error is
    at most (1 + C) times the discretisation error, C from the V-cycle's contraction)."""
    levels = om.hierarchy(n0, refine, p)
    lev = levels[-1]
    mg = solvers.MGHierarchy(levels)
    b = assemble.load_vector(lev, fem_inputs.sin3_f, 2 * p + 4)
    b[lev.boundary] = 0
    u_fmg = mg.fmg(b)
    u_h = solvers.direct_solve(mg.levels[-1].A, b)
    e_fmg = assemble.l2_error(lev, u_fmg, fem_inputs.sin3_u, 2 * p + 4)
    e_h = assemble.l2_error(lev, u_h, fem_inputs.sin3_u, 2 * p + 4)
    assert e_fmg <= 2.0 * e_h, (e_fmg, e_h)
    # its distance from the discrete solution is of the order of the discretisation error
    d = assemble.l2_error(lev, u_fmg - u_h, lambda x: np.zeros(len(x)), 2 * p + 4)
    assert d <= 1.5 * e_h, (d, e_h)


def test_fmg_linear_and_exact_on_one_level():
    levels = om.hierarchy(2, 1, 2, fem_inputs.jitter_offsets(2, 0.1))
    mg = solvers.MGHierarchy(levels)
    lev = levels[-1]
    b1 = fem_inputs.uniform_vector(lev.n_dofs, 0)
    b2 = fem_inputs.uniform_vector(lev.n_dofs, 7)
    b1[lev.boundary] = 0
    b2[lev.boundary] = 0
    lhs = mg.fmg(2.5 * b1 + b2)
    rhs = 2.5 * mg.fmg(b1) + mg.fmg(b2)
    assert np.linalg.norm(lhs - rhs) <= 1e-12 * np.linalg.norm(rhs)
    one = solvers.MGHierarchy(levels[:1])
    bc = fem_inputs.uniform_vector(levels[0].n_dofs, 3)
    bc[levels[0].boundary] = 0
    x = one.fmg(bc)
    assert np.linalg.norm(one.levels[0].A @ x - bc) <= 1e-12 * np.linalg.norm(bc)
