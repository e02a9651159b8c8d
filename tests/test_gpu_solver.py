"""GPU parity of the multigrid-CG solver against the oracle, through the C ABI.

* One FP64 V-cycle against the oracle's V-cycle with the same lambda_max (1e-12): exercises the
  Chebyshev smoother, transfers, rediscretised coefficient and exact coarse solve together; two-,
  three- and four-level cycles.
* Solutions to rtol 1e-10 against the oracle's reference solution (1e-8), FP64 and mixed.
* Jacobi-CG on the P1 8^3 workload (iteration bound 60 for 1e-10).
* Nested coarse solve (FP64 MG-PCG over the levels below the coarsest level used): one V-cycle
  against the oracle's V-cycle on the truncated hierarchy (exact coarse solve) to 1e-9, and
  solutions against the oracle's reference solution (1e-8), FP64 and mixed.
* Failure handling: max_it reached, NaN right-hand side, negative coefficient, bad arguments.
* Determinism and warm start.
* Mixed precision keeps the coarse solve in FP64 (the FP32-stored inverse only on request).
* The dense coarse inverse alone (full multigrid on one level is the coarse solve) against the
  oracle's direct solve to FP64 accuracy, at sizes with several 256-wide pivot blocks and ragged
  tails.
"""
import numpy as np
import pytest

import fem_inputs
from oracle import assemble, solvers
from tests.gpu_util import banner, make_pair, oracle_A, rel

torch = pytest.importorskip("torch")


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda:0")


def _rhs(lev):
    b = assemble.mass(lev) @ fem_inputs.sin3_f(lev.dof_xyz())
    b[lev.boundary] = 0
    return b


@pytest.mark.gpu
@pytest.mark.parametrize("n0,r,p,jit,kvar", [(2, 2, 2, 0.1, True), (2, 2, 1, 0.0, False), (2, 1, 3, 0.1, True),
                                             (3, 1, 2, 0.0, True),
                                             # four-level cycles, as the P3 k = exp(g) workload runs
                                             (1, 3, 2, 0.1, True), (1, 3, 3, 0.0, True)])
def test_vcycle_matches_oracle(n0, r, p, jit, kvar):
    banner(f"vcycle n0={n0} r={r} p={p} kvar={kvar}")
    from paper_2104_08012_amd import fem
    mesh, levels = make_pair(n0, r, p, jit)
    k = fem_inputs.k_exp_fourier(levels[-1].vert_xyz) if kvar else None
    omg = solvers.MGHierarchy(levels, k)
    lm = [0.0] + [L.lmax for L in omg.levels[1:]]
    opts = fem.SolveOptions(lambda_max=lm)
    S = fem.Solver(mesh, opts).setup(_t(k) if kvar else None)
    x = fem_inputs.uniform_vector(levels[-1].n_dofs, 0)
    x[levels[-1].boundary] = 0
    z = S.vcycle(_t(x))
    torch.cuda.synchronize()
    assert rel(z.cpu().numpy(), omg.vcycle(x)) <= 1e-12


@pytest.mark.gpu
@pytest.mark.parametrize("n0,r,p,jit,kvar,prec", [
    (2, 2, 2, 0.1, False, "fp64"), (2, 2, 2, 0.1, True, "mixed"), (2, 2, 1, 0.0, False, "mixed"),
    (2, 1, 3, 0.1, True, "fp64"), (2, 1, 3, 0.0, True, "mixed"), (4, 1, 2, 0.15, True, "fp64")])
def test_solution_parity(n0, r, p, jit, kvar, prec):
    banner(f"solve n0={n0} r={r} p={p} kvar={kvar} {prec}")
    from paper_2104_08012_amd import fem
    mesh, levels = make_pair(n0, r, p, jit)
    lev = levels[-1]
    k = fem_inputs.k_exp_fourier(lev.vert_xyz) if kvar else None
    A = assemble.apply_bc(assemble.stiffness(lev, k), lev.boundary)
    b = _rhs(lev)
    u_ref = solvers.direct_solve(A, b, rtol=1e-14)
    S = fem.Solver(mesh, fem.SolveOptions(rtol=1e-10, precision=prec)).setup(_t(k) if kvar else None)
    u, res = S.solve(_t(b))
    torch.cuda.synchronize()
    assert res.rel_residual_true <= 1e-10
    assert rel(u.cpu().numpy(), u_ref) <= 1e-8
    assert res.iterations <= 40


@pytest.mark.gpu
@pytest.mark.parametrize("p,kvar", [(2, True), (1, False)])
def test_nested_coarse_vcycle(p, kvar):
    banner(f"nested vcycle p={p} kvar={kvar}")
    from paper_2104_08012_amd import fem
    mesh, levels = make_pair(2, 2, p, 0.1)
    k = fem_inputs.k_exp_fourier(levels[-1].vert_xyz) if kvar else None
    omg = solvers.MGHierarchy(levels[1:], k)      # exact solve on level 1
    lm = [0.0, 0.0, omg.levels[1].lmax]
    opts = fem.SolveOptions(lambda_max=lm, n_levels_used=2, coarse_method="nested", coarse_rtol=1e-13)
    S = fem.Solver(mesh, opts).setup(_t(k) if kvar else None)
    x = fem_inputs.uniform_vector(levels[-1].n_dofs, 0)
    x[levels[-1].boundary] = 0
    z = S.vcycle(_t(x))
    torch.cuda.synchronize()
    assert rel(z.cpu().numpy(), omg.vcycle(x)) <= 1e-9


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_nested_coarse_solution(prec):
    banner(f"nested solve p=2 {prec}")
    from paper_2104_08012_amd import fem
    mesh, levels = make_pair(2, 2, 2, 0.1)
    lev = levels[-1]
    k = fem_inputs.k_exp_fourier(lev.vert_xyz)
    A = assemble.apply_bc(assemble.stiffness(lev, k), lev.boundary)
    b = _rhs(lev)
    u_ref = solvers.direct_solve(A, b, rtol=1e-14)
    opts = fem.SolveOptions(rtol=1e-10, precision=prec, n_levels_used=2, coarse_method="nested")
    S = fem.Solver(mesh, opts).setup(_t(k))
    u, res = S.solve(_t(b))
    torch.cuda.synchronize()
    assert res.rel_residual_true <= 1e-10
    assert rel(u.cpu().numpy(), u_ref) <= 1e-8
    assert res.coarse_iterations > 0
    # the same system with the dense coarse inverse on level 1
    Sd = fem.Solver(mesh, fem.SolveOptions(rtol=1e-10, precision=prec, n_levels_used=2,
                                           coarse_method="dense")).setup(_t(k))
    ud, resd = Sd.solve(_t(b))
    torch.cuda.synchronize()
    assert resd.coarse_iterations == 0
    assert rel(u.cpu().numpy(), ud.cpu().numpy()) <= 1e-8


@pytest.mark.gpu
def test_nested_needs_a_lower_level():
    banner("nested on level 0 rejected")
    from paper_2104_08012_amd import fem
    from paper_2104_08012_amd._lib import FemError
    mesh, _ = make_pair(2, 1, 1, 0.0)
    with pytest.raises(FemError):
        fem.Solver(mesh, fem.SolveOptions(coarse_method="nested"))


@pytest.mark.gpu
def test_jacobi_cg_p1_8():
    banner("jacobi cg p1 8^3")
    from paper_2104_08012_amd import fem
    mesh, levels = make_pair(8, 0, 1, 0.0)
    lev = levels[0]
    A = assemble.apply_bc(assemble.stiffness(lev), lev.boundary)
    b = assemble.load_vector(lev, fem_inputs.sin3_f, 6)
    b[lev.boundary] = 0
    S = fem.Solver(mesh, fem.SolveOptions(rtol=1e-10, preconditioner="jacobi")).setup()
    u, res = S.solve(_t(b))
    assert res.iterations <= 60
    assert res.rel_residual_true <= 1e-10
    assert rel(u.cpu().numpy(), solvers.direct_solve(A, b)) <= 1e-8


@pytest.mark.gpu
def test_failure_modes():
    banner("failure modes")
    from paper_2104_08012_amd import fem
    from paper_2104_08012_amd._lib import FEM_ERR_BREAKDOWN, FEM_WARN_NOT_CONVERGED, FemError
    mesh, levels = make_pair(2, 2, 2, 0.0)
    lev = levels[-1]
    b = _t(_rhs(lev))
    S = fem.Solver(mesh, fem.SolveOptions(rtol=1e-12, max_it=1)).setup()
    x, res = S.solve(b, allow_not_converged=True)
    assert res.status == FEM_WARN_NOT_CONVERGED and res.iterations == 1
    with pytest.raises(FemError) as e:
        S.solve(b)
    assert e.value.status == FEM_WARN_NOT_CONVERGED
    bn = b.clone()
    bn[5] = float("nan")
    with pytest.raises(FemError) as e:
        S.solve(bn)
    assert e.value.status == FEM_ERR_BREAKDOWN
    kneg = -torch.ones(lev.n_vertices, dtype=torch.float64, device="cuda:0")
    S2 = fem.Solver(mesh, fem.SolveOptions(rtol=1e-10, preconditioner="jacobi")).setup(kneg)
    with pytest.raises(FemError) as e:
        S2.solve(b)
    assert e.value.status == FEM_ERR_BREAKDOWN
    with pytest.raises(FemError):
        fem.Solver(mesh, fem.SolveOptions(rtol=-1.0))


@pytest.mark.gpu
def test_determinism_and_warm_start():
    banner("determinism / warm start")
    from paper_2104_08012_amd import fem
    mesh, levels = make_pair(2, 2, 2, 0.1)
    lev = levels[-1]
    b = _t(_rhs(lev))
    S = fem.Solver(mesh, fem.SolveOptions(rtol=1e-10)).setup()
    u1, r1 = S.solve(b)
    u2, r2 = S.solve(b)
    assert torch.equal(u1, u2) and r1.iterations == r2.iterations and r1.history == r2.history
    S4 = fem.Solver(mesh, fem.SolveOptions(rtol=1e-4)).setup()
    x, ra = S4.solve(b)
    x, rb = S.solve(b, x=x)
    assert rb.rel_residual_true <= 1e-10 and rb.iterations < r1.iterations


@pytest.mark.gpu
@pytest.mark.parametrize("p,kvar,used", [(2, True, 0), (1, False, 0), (2, False, 2)])
def test_fmg_matches_oracle(p, kvar, used):
    """One full-multigrid cycle against the oracle's (same lambda_max on every level): FP64 to
    1e-10; the mixed-precision cycle within FP32 rounding of it; on the truncated hierarchy
    (used = 2) the coarse level is the nested solve's."""
    banner(f"fmg p={p} kvar={kvar} used={used}")
    from paper_2104_08012_amd import fem
    mesh, levels = make_pair(2, 2, p, 0.1)
    lev = levels[-1]
    k = fem_inputs.k_exp_fourier(lev.vert_xyz) if kvar else None
    sub = levels if used == 0 else levels[-used:]
    omg = solvers.MGHierarchy(sub, k)
    lm = [0.0] * (len(levels) - len(sub)) + [0.0] + [L.lmax for L in omg.levels[1:]]
    b = _rhs(lev)
    x_ref = omg.fmg(b)
    extra = dict(n_levels_used=used, coarse_method="nested", coarse_rtol=1e-13) if used else {}
    S = fem.Solver(mesh, fem.SolveOptions(lambda_max=lm, **extra)).setup(_t(k) if kvar else None)
    x, res = S.fmg(_t(b))
    torch.cuda.synchronize()
    assert rel(x.cpu().numpy(), x_ref) <= (1e-9 if used else 1e-10)
    r_ref = np.linalg.norm(b - omg.levels[-1].A @ x_ref) / np.linalg.norm(b)
    assert abs(res.rel_residual_true - r_ref) <= 1e-6 * r_ref
    Sm = fem.Solver(mesh, fem.SolveOptions(lambda_max=lm, precision="mixed", **extra)).setup(_t(k) if kvar else None)
    xm, _ = Sm.fmg(_t(b))
    torch.cuda.synchronize()
    assert rel(xm.cpu().numpy(), x_ref) <= 1e-5


@pytest.mark.gpu
@pytest.mark.parametrize("p", [1, 2])
def test_smallest_meshes_and_zero_rhs(p):
    """Degenerate cases: one cube (P1: no interior dof), a 1-cube coarse level under one
    refinement (dense coarse block of size 0 for P1), a zero right-hand side, and full multigrid
    on a single level (the exact coarse solve alone)."""
    banner(f"smallest meshes p={p}")
    from paper_2104_08012_amd import fem
    mesh1, lv1 = make_pair(1, 0, p, 0.0)
    x = fem_inputs.uniform_vector(lv1[0].n_dofs, 0)
    y = mesh1.apply(_t(x), level=0)
    torch.cuda.synchronize()
    assert rel(y.cpu().numpy(), oracle_A(lv1[0]) @ x) <= 1e-12
    S1 = fem.Solver(mesh1, fem.SolveOptions(rtol=1e-12)).setup()
    b1 = _rhs(lv1[0])
    u1, r1 = S1.fmg(_t(b1))
    torch.cuda.synchronize()
    assert rel(u1.cpu().numpy(), solvers.direct_solve(oracle_A(lv1[0]), b1)) <= 1e-12 or np.linalg.norm(b1) == 0
    mesh, levels = make_pair(1, 1, p, 0.0)
    lev = levels[-1]
    b = _rhs(lev)
    S = fem.Solver(mesh, fem.SolveOptions(rtol=1e-12)).setup()
    u, res = S.solve(_t(b))
    torch.cuda.synchronize()
    assert rel(u.cpu().numpy(), solvers.direct_solve(oracle_A(lev), b)) <= 1e-10
    z, rz = S.solve(torch.zeros(lev.n_dofs, dtype=torch.float64, device="cuda:0"))
    torch.cuda.synchronize()
    assert rz.iterations == 0 and float(z.abs().max()) == 0.0


@pytest.mark.gpu
def test_mixed_precision_coarse_solve_is_fp64():
    """In mixed precision the coarse solve stays FP64 (Section 4's direct coarse solve; the FP32
    part of the method is the smoother and the transfers): full multigrid on one level is the
    coarse solve alone, so the mixed solver's result equals the oracle's direct solve to FP64
    accuracy.  The FP32-stored inverse (coarse_method "dense_f32") is an explicit option and
    agrees only to FP32 accuracy."""
    banner("mixed coarse solve FP64 / dense_f32")
    from paper_2104_08012_amd import fem
    mesh, levels = make_pair(4, 1, 2, 0.1)
    lev = levels[-1]
    k = fem_inputs.k_exp_fourier(lev.vert_xyz)
    A = assemble.apply_bc(assemble.stiffness(lev, k), lev.boundary)
    b = _rhs(lev)
    u_ref = solvers.direct_solve(A, b, rtol=1e-14)
    for cm, tol in (("auto", 1e-11), ("dense", 1e-11), ("dense_f32", 1e-5)):
        S = fem.Solver(mesh, fem.SolveOptions(precision="mixed", n_levels_used=1, coarse_method=cm)).setup(_t(k))
        u, _ = S.fmg(_t(b))
        torch.cuda.synchronize()
        assert rel(u.cpu().numpy(), u_ref) <= tol, cm
    # and the outer solve with the FP32-stored inverse still reaches the FP64 residual
    S = fem.Solver(mesh, fem.SolveOptions(rtol=1e-10, precision="mixed", coarse_method="dense_f32")).setup(_t(k))
    u, res = S.solve(_t(b))
    torch.cuda.synchronize()
    assert res.rel_residual_true <= 1e-10 and rel(u.cpu().numpy(), u_ref) <= 1e-8


@pytest.mark.gpu
@pytest.mark.parametrize("n0,r,p,jit,kvar", [(2, 1, 3, 0.1, True),     # 11^3 = 1331 interior: 5 blocks + 51
                                             (10, 1, 1, 0.1, False),   # 19^3 = 6859: 26 blocks + 203
                                             (9, 0, 1, 0.1, True),     # 8^3 = 512: exactly 2 blocks
                                             (35, 0, 1, 0.1, False)])  # 34^3 = 39304, near the 40000 limit
def test_dense_coarse_inverse_is_exact(n0, r, p, jit, kvar):
    banner(f"dense coarse inverse n0={n0} r={r} p={p}")
    from paper_2104_08012_amd import fem
    mesh, levels = make_pair(n0, r, p, jit)
    lev = levels[-1]
    k = fem_inputs.k_exp_fourier(lev.vert_xyz) if kvar else None
    A = assemble.apply_bc(assemble.stiffness(lev, k), lev.boundary)
    b = _rhs(lev)
    u_ref = solvers.direct_solve(A, b, rtol=1e-14)
    S = fem.Solver(mesh, fem.SolveOptions(n_levels_used=1, coarse_method="dense")).setup(_t(k) if kvar else None)
    u, _ = S.fmg(_t(b))
    torch.cuda.synchronize()
    assert rel(u.cpu().numpy(), u_ref) <= 1e-11
    # a second, independent setup gives the same inverse bit for bit (fixed reduction orders)
    S2 = fem.Solver(mesh, fem.SolveOptions(n_levels_used=1, coarse_method="dense")).setup(_t(k) if kvar else None)
    u2, _ = S2.fmg(_t(b))
    torch.cuda.synchronize()
    assert torch.equal(u, u2)
