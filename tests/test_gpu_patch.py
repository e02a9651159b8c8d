"""GPU parity of the additive vertex-star patch preconditioner (P2 and P3) against the oracle
(oracle/patch.py), through the C ABI.

* FP64: max |z - z_ref| <= 1e-11 max |z_ref|.  The star inverses come from Gauss-Jordan
  elimination of 15x15 symmetric positive definite blocks (condition numbers below 1e3 on these
  meshes), so their entries carry relative errors of order cond * 15 * 2^-53 ~ 2e-12; the oracle
  inverts the same blocks with LAPACK.
* FP32 storage (inverses computed in FP64, rounded once; residual and sums in FP32):
  max |z - z_ref| <= 2e-5 max |z_ref| (15-term sums of FP32 products, cond below 1e3).
* Boundary entries pass through bit-exactly; repeated applications are bitwise equal.
* Meshes span the brick sizes of the cell order (B = 4, 2, 1), several bricks per direction,
  jittered vertices with a P1 coefficient k, a level of a refined hierarchy, and the degenerate
  one-cube mesh whose only interior dof lies in two stars.
* At the 64^3 workload's finest level (2,146,689 dofs) the sampled check is by properties that
  hold at any size: symmetry (r2 . B r1 = r1 . B r2) and positivity of r . B r, boundary
  pass-through.
* P3 (65-dof stars, 2145 packed inverse entries per vertex): the same cases on small meshes,
  FP64 1e-11 and FP32 NS kappa 2^-24 of max |z_ref| (kappa the largest condition number of the
  oracle's star matrices, about 20 here: the bound of 65-term FP32 sums of rounded entries);
  the 48^3 k = exp(g) finest level by sampled dofs against the oracle's one-dof-at-a-time
  evaluation and by symmetry and positivity; a patch-smoothed V-cycle and MG-CG solutions
  against the oracle's.
"""
import numpy as np
import pytest

import fem_inputs
from oracle import patch
from oracle import patch as op
from tests.gpu_util import banner, make_pair, oracle_A

torch = pytest.importorskip("torch")


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda:0")


@pytest.mark.gpu
@pytest.mark.parametrize("n,nref,level,jit,kvar", [
    (1, 0, 0, 0.0, False),
    (4, 0, 0, 0.0, False),
    (3, 0, 0, 0.15, True),
    (6, 0, 0, 0.1, True),
    (8, 0, 0, 0.15, True),
    (2, 1, 1, 0.1, True),
    (2, 1, 0, 0.1, True),
])
def test_patch_apply_matches_oracle(n, nref, level, jit, kvar):
    banner(f"patch n={n} nref={nref} level={level} jit={jit} kvar={kvar}")
    from paper_2104_08012_amd import fem
    mesh, levels = make_pair(n, nref, 2, jit)
    lev = levels[level]
    k = fem_inputs.k_exp_fourier(lev.vert_xyz) if kvar else None
    A = oracle_A(lev, k)
    pts = patch.star_patches(lev)
    inv = patch.patch_inverses(A, pts)
    r = fem_inputs.uniform_vector(lev.n_dofs, seed=0)
    zr = patch.apply_patch_pc(pts, inv, lev.boundary, r)
    for dtype, tol in ((torch.float64, 1e-11), (torch.float32, 2e-5)):
        pc = fem.PatchPreconditioner(mesh, level, _t(k) if kvar else None, dtype=dtype)
        rt = _t(r, dtype)
        z1 = pc.apply(rt)
        z2 = pc.apply(rt)
        torch.cuda.synchronize()
        z = z1.double().cpu().numpy()
        assert np.abs(z - zr).max() <= tol * np.abs(zr).max()
        assert torch.equal(z1, z2)
        assert np.array_equal(z[lev.boundary], rt.double().cpu().numpy()[lev.boundary])


@pytest.mark.gpu
def test_patch_properties_at_workload_size():
    banner("patch properties P2 64^3 finest level")
    from paper_2104_08012_amd import fem
    mesh = fem.Mesh(16, 2, 2, device="cuda:0")
    N = mesh.n_dofs(-1)
    assert N == 129 ** 3
    bnd_lat = np.zeros((129, 129, 129), dtype=bool)
    bnd_lat[[0, -1], :, :] = True
    bnd_lat[:, [0, -1], :] = True
    bnd_lat[:, :, [0, -1]] = True
    bnd = bnd_lat.ravel()
    pc = fem.PatchPreconditioner(mesh, -1, None, dtype=torch.float64)
    r1 = fem_inputs.uniform_vector(N, seed=0)
    r2 = fem_inputs.uniform_vector(N, seed=1)
    r1[bnd] = 0.0
    r2[bnd] = 0.0
    z1 = pc.apply(_t(r1)).cpu().numpy()
    z2 = pc.apply(_t(r2)).cpu().numpy()
    a, b = r2 @ z1, r1 @ z2
    assert abs(a - b) <= 1e-12 * np.sqrt(abs(r1 @ z1) * abs(r2 @ z2))
    assert r1 @ z1 > 0 and r2 @ z2 > 0
    assert np.all(z1[bnd] == 0.0)
    rb = fem_inputs.uniform_vector(N, seed=2)
    zb = pc.apply(_t(rb)).cpu().numpy()
    assert np.array_equal(zb[bnd], rb[bnd])


@pytest.mark.gpu
def test_patch_argument_errors():
    banner("patch argument errors")
    from paper_2104_08012_amd import fem
    from paper_2104_08012_amd._lib import FEM_ERR_UNSUPPORTED, lib
    import ctypes as C
    mesh1 = fem.Mesh(4, 0, 1, device="cuda:0")
    nb = C.c_size_t()
    assert lib().fem_patch_bytes(mesh1.handle, 0, 0, C.byref(nb)) == FEM_ERR_UNSUPPORTED
    mesh = fem.Mesh(4, 0, 2, device="cuda:0")
    pc = fem.PatchPreconditioner(mesh, 0)
    r = torch.zeros(mesh.n_dofs(0), dtype=torch.float64, device="cuda:0")
    with pytest.raises(Exception):
        pc.apply(r, out=r)
    with pytest.raises(ValueError):
        pc.apply(r.float())


def _rhs(lev):
    from oracle import assemble
    b = assemble.mass(lev) @ fem_inputs.sin3_f(lev.dof_xyz())
    b[lev.boundary] = 0
    return b


@pytest.mark.gpu
@pytest.mark.parametrize("n0,r,jit,kvar", [(2, 2, 0.1, True), (3, 1, 0.0, True), (2, 1, 0.0, False)])
def test_patch_smoothed_vcycle_matches_oracle(n0, r, jit, kvar):
    # one FP64 V-cycle with the patch-preconditioned Chebyshev smoother against the oracle's, same
    # lambda_max per level: 1e-11 (the 15x15 star inverses carry ~2e-12 relative errors)
    banner(f"patch vcycle n0={n0} r={r} kvar={kvar}")
    from oracle import solvers
    from paper_2104_08012_amd import fem
    from tests.gpu_util import rel
    mesh, levels = make_pair(n0, r, 2, jit)
    k = fem_inputs.k_exp_fourier(levels[-1].vert_xyz) if kvar else None
    omg = solvers.MGHierarchy(levels, k, smoother="patch")
    lm = [0.0] + [L.lmax for L in omg.levels[1:]]
    S = fem.Solver(mesh, fem.SolveOptions(lambda_max=lm, smoother="patch")).setup(_t(k) if kvar else None)
    x = fem_inputs.uniform_vector(levels[-1].n_dofs, 0)
    x[levels[-1].boundary] = 0
    z = S.vcycle(_t(x))
    torch.cuda.synchronize()
    assert rel(z.cpu().numpy(), omg.vcycle(x)) <= 1e-11


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_patch_smoothed_solution_parity(prec):
    banner(f"patch-smoothed solve {prec}")
    from oracle import assemble, solvers
    from paper_2104_08012_amd import fem
    from tests.gpu_util import rel
    mesh, levels = make_pair(2, 2, 2, 0.1)
    lev = levels[-1]
    k = fem_inputs.k_exp_fourier(lev.vert_xyz)
    A = assemble.apply_bc(assemble.stiffness(lev, k), lev.boundary)
    b = _rhs(lev)
    u_ref = solvers.direct_solve(A, b, rtol=1e-14)
    S = fem.Solver(mesh, fem.SolveOptions(rtol=1e-10, precision=prec, smoother="patch")).setup(_t(k))
    u, res = S.solve(_t(b))
    Sj = fem.Solver(mesh, fem.SolveOptions(rtol=1e-10, precision=prec)).setup(_t(k))
    _, resj = Sj.solve(_t(b))
    torch.cuda.synchronize()
    print(f"iterations patch {res.iterations} jacobi {resj.iterations}", flush=True)
    assert res.rel_residual_true <= 1e-10
    assert rel(u.cpu().numpy(), u_ref) <= 1e-8
    assert res.iterations <= resj.iterations
    # the CG-Lanczos estimate on the finest level lies inside the spectrum of B A and close to its top
    if prec == "fp64":
        from oracle import patch as op
        pts = op.star_patches(lev)
        inv = op.patch_inverses(A, pts)
        Bd = np.stack([op.apply_patch_pc(pts, inv, lev.boundary, e) for e in np.eye(lev.n_dofs)], axis=1)
        lam = np.max(np.linalg.eigvals(Bd @ A.toarray()).real)
        est = res.lambda_max[len(levels) - 1]
        assert 0.9 * lam <= est <= lam * (1 + 1e-9)


@pytest.mark.gpu
def test_patch_smoother_needs_degree_2_or_3():
    banner("patch smoother degree check")
    from paper_2104_08012_amd import fem
    from paper_2104_08012_amd._lib import FemError
    mesh = fem.Mesh(2, 1, 1, device="cuda:0")
    with pytest.raises(FemError):
        fem.Solver(mesh, fem.SolveOptions(smoother="patch"))


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_patch_smoother_with_nested_coarse_solve(prec):
    # outer cycle on the two finest levels with patch smoothing; its coarse level is solved by the
    # nested FP64 MG-PCG (Jacobi-smoothed) over the levels below
    banner(f"patch smoother + nested coarse {prec}")
    from oracle import assemble, solvers
    from paper_2104_08012_amd import fem
    from tests.gpu_util import rel
    mesh, levels = make_pair(2, 2, 2, 0.1)
    lev = levels[-1]
    k = fem_inputs.k_exp_fourier(lev.vert_xyz)
    A = assemble.apply_bc(assemble.stiffness(lev, k), lev.boundary)
    b = _rhs(lev)
    u_ref = solvers.direct_solve(A, b, rtol=1e-14)
    opts = fem.SolveOptions(rtol=1e-10, precision=prec, smoother="patch", n_levels_used=2,
                            coarse_method="nested")
    S = fem.Solver(mesh, opts).setup(_t(k))
    u, res = S.solve(_t(b))
    torch.cuda.synchronize()
    assert res.rel_residual_true <= 1e-10
    assert rel(u.cpu().numpy(), u_ref) <= 1e-8
    assert res.coarse_iterations > 0


@pytest.mark.gpu
@pytest.mark.parametrize("kvar", [False, True])
def test_patch_sampled_parity_at_workload_size(kvar):
    # the 64^3 P2 finest level in the launch configuration the benchmark times, against the
    # oracle's one-dof-at-a-time evaluation on sampled dofs: random interior dofs, dofs next to
    # the boundary and at the corners, and boundary dofs
    banner(f"patch sampled parity 64^3 kvar={kvar}")
    from oracle import mesh as om
    from paper_2104_08012_amd import fem
    mesh = fem.Mesh(16, 2, 2, device="cuda:0")
    lev = om.hierarchy(16, 2, 2)[-1]
    L = 129
    k = fem_inputs.k_exp_fourier(lev.vert_xyz) if kvar else None
    r = fem_inputs.uniform_vector(lev.n_dofs, seed=0)
    rng = np.random.default_rng(11)
    pts = [(1, 1, 1), (127, 127, 127), (1, 2, 2), (2, 1, 127), (64, 64, 64), (63, 65, 64), (1, 64, 127),
           (0, 5, 7), (128, 64, 3)]
    sample = [i + L * (j + L * kk) for i, j, kk in pts]
    sample += rng.integers(0, lev.n_dofs, 40).tolist()
    face = rng.integers(1, 128, (20, 3))
    face[:, 0] = rng.choice([1, 2, 126, 127], 20)
    sample += [int(i + L * (j + L * kk)) for i, j, kk in face]
    sample = np.array(sample)
    zr = op.patch_pc_at(lev, k, r, sample)
    for dtype, tol in ((torch.float64, 1e-11), (torch.float32, 2e-5)):
        pc = fem.PatchPreconditioner(mesh, -1, _t(k) if kvar else None, dtype=dtype)
        z = pc.apply(_t(r, dtype)).double().cpu().numpy()[sample]
        assert np.abs(z - zr).max() <= tol * np.abs(zr).max()


@pytest.mark.gpu
def test_patch_smoothed_fmg_matches_oracle():
    # one full-multigrid cycle (Listing 2's solver configuration) with the patch-preconditioned
    # smoother against the oracle's, same lambda_max: FP64 1e-10, mixed within FP32 rounding
    banner("patch-smoothed fmg")
    from oracle import solvers
    from paper_2104_08012_amd import fem
    from tests.gpu_util import rel
    mesh, levels = make_pair(2, 2, 2, 0.1)
    lev = levels[-1]
    k = fem_inputs.k_exp_fourier(lev.vert_xyz)
    omg = solvers.MGHierarchy(levels, k, smoother="patch")
    lm = [0.0] + [L.lmax for L in omg.levels[1:]]
    b = _rhs(lev)
    x_ref = omg.fmg(b)
    for prec, tol in (("fp64", 1e-10), ("mixed", 1e-5)):
        S = fem.Solver(mesh, fem.SolveOptions(lambda_max=lm, precision=prec, smoother="patch")).setup(_t(k))
        x, _ = S.fmg(_t(b))
        torch.cuda.synchronize()
        assert rel(x.cpu().numpy(), x_ref) <= tol


def _p3_tolerances(A, pts):
    kappa = max(np.linalg.cond(A[i][:, i].toarray()) for i in pts if i.size)
    return 1e-11, max(2e-5, 65 * kappa * 2.0 ** -24)


@pytest.mark.gpu
@pytest.mark.parametrize("n,nref,level,jit,kvar", [
    (1, 0, 0, 0.0, False),
    (2, 0, 0, 0.0, False),
    (3, 0, 0, 0.15, True),
    (4, 0, 0, 0.1, True),
    (6, 0, 0, 0.1, True),
    (2, 1, 1, 0.1, True),
    (2, 1, 0, 0.1, True),
])
def test_p3_patch_apply_matches_oracle(n, nref, level, jit, kvar):
    banner(f"P3 patch n={n} nref={nref} level={level} jit={jit} kvar={kvar}")
    from paper_2104_08012_amd import fem
    mesh, levels = make_pair(n, nref, 3, jit)
    lev = levels[level]
    k = fem_inputs.k_exp_fourier(lev.vert_xyz) if kvar else None
    A = oracle_A(lev, k)
    pts = patch.star_patches(lev)
    inv = patch.patch_inverses(A, pts)
    tol64, tol32 = _p3_tolerances(A.tocsr(), pts)
    r = fem_inputs.uniform_vector(lev.n_dofs, seed=0)
    zr = patch.apply_patch_pc(pts, inv, lev.boundary, r)
    for dtype, tol in ((torch.float64, tol64), (torch.float32, tol32)):
        pc = fem.PatchPreconditioner(mesh, level, _t(k) if kvar else None, dtype=dtype)
        rt = _t(r, dtype)
        z1 = pc.apply(rt)
        z2 = pc.apply(rt)
        torch.cuda.synchronize()
        z = z1.double().cpu().numpy()
        err = np.abs(z - zr).max() / np.abs(zr).max()
        print(f"[patch3] {dtype}: {err:.2e} (tol {tol:.1e})", flush=True)
        assert err <= tol
        assert torch.equal(z1, z2)
        assert np.array_equal(z[lev.boundary], rt.double().cpu().numpy()[lev.boundary])


@pytest.mark.gpu
def test_p3_patch_at_workload_size():
    # the 48^3 P3 finest level with k = exp(g) (3,048,625 dofs, 117,649 stars): sampled dofs
    # (vertices, edge and face dofs, next to the boundary, on brick planes, random) against the
    # oracle's one-dof-at-a-time evaluation; symmetry and positivity; boundary pass-through
    banner("P3 patch 48^3 k=exp(g): sampled parity and properties")
    from oracle import mesh as om
    from paper_2104_08012_amd import fem
    mesh = fem.Mesh(6, 3, 3, device="cuda:0")
    lev = om.hierarchy(6, 3, 3)[-1]
    L = 145
    k = fem_inputs.k_exp_fourier(lev.vert_xyz)
    kt = _t(k)
    r = fem_inputs.uniform_vector(lev.n_dofs, seed=0)
    rng = np.random.default_rng(21)
    pts = [(3, 3, 3), (1, 1, 1), (2, 1, 1), (1, 2, 3), (141, 143, 142), (72, 72, 72), (73, 71, 72), (12, 13, 14),
           (36, 37, 1), (4, 5, 5), (0, 5, 7), (144, 64, 3), (24, 25, 26), (143, 1, 72)]
    sample = [i + L * (j + L * kk) for i, j, kk in pts]
    sample += rng.integers(0, lev.n_dofs, 24).tolist()
    sample = np.array(sample)
    print("[patch3] oracle sampled evaluation ...", flush=True)
    zr = op.patch_pc_at(lev, k, r, sample)
    pc64 = fem.PatchPreconditioner(mesh, -1, kt, dtype=torch.float64)
    z = pc64.apply(_t(r)).cpu().numpy()[sample]
    err = np.abs(z - zr).max() / np.abs(zr).max()
    print(f"[patch3] fp64 sampled err {err:.2e}", flush=True)
    assert err <= 1e-11
    pc32 = fem.PatchPreconditioner(mesh, -1, kt, dtype=torch.float32)
    z32 = pc32.apply(_t(r, torch.float32)).double().cpu().numpy()[sample]
    err32 = np.abs(z32 - zr).max() / np.abs(zr).max()
    print(f"[patch3] fp32 sampled err {err32:.2e}", flush=True)
    assert err32 <= 1e-4
    del pc32
    bnd = lev.boundary
    r1 = fem_inputs.uniform_vector(lev.n_dofs, seed=1)
    r2 = fem_inputs.uniform_vector(lev.n_dofs, seed=2)
    r1[bnd] = 0.0
    r2[bnd] = 0.0
    z1 = pc64.apply(_t(r1)).cpu().numpy()
    z2 = pc64.apply(_t(r2)).cpu().numpy()
    a, b = r2 @ z1, r1 @ z2
    assert abs(a - b) <= 1e-12 * np.sqrt(abs(r1 @ z1) * abs(r2 @ z2))
    assert r1 @ z1 > 0 and r2 @ z2 > 0
    assert np.all(z1[bnd] == 0.0)
    zb = pc64.apply(_t(r)).cpu().numpy()
    assert np.array_equal(zb[bnd], r[bnd])


@pytest.mark.gpu
@pytest.mark.parametrize("n0,r,jit,kvar", [(2, 1, 0.1, True), (1, 2, 0.0, True), (2, 1, 0.0, False)])
def test_p3_patch_smoothed_vcycle_matches_oracle(n0, r, jit, kvar):
    banner(f"P3 patch vcycle n0={n0} r={r} kvar={kvar}")
    from oracle import solvers
    from paper_2104_08012_amd import fem
    from tests.gpu_util import rel
    mesh, levels = make_pair(n0, r, 3, jit)
    k = fem_inputs.k_exp_fourier(levels[-1].vert_xyz) if kvar else None
    omg = solvers.MGHierarchy(levels, k, smoother="patch")
    lm = [0.0] + [L.lmax for L in omg.levels[1:]]
    S = fem.Solver(mesh, fem.SolveOptions(lambda_max=lm, smoother="patch")).setup(_t(k) if kvar else None)
    x = fem_inputs.uniform_vector(levels[-1].n_dofs, 0)
    x[levels[-1].boundary] = 0
    z = S.vcycle(_t(x))
    torch.cuda.synchronize()
    assert rel(z.cpu().numpy(), omg.vcycle(x)) <= 1e-11


@pytest.mark.gpu
@pytest.mark.parametrize("prec,n0,r", [("fp64", 1, 1), ("mixed", 1, 1), ("fp64", 2, 1), ("mixed", 2, 1)])
def test_p3_patch_smoothed_solution_parity(prec, n0, r):
    banner(f"P3 patch-smoothed solve {prec} n0={n0} r={r}")
    from oracle import assemble, solvers
    from paper_2104_08012_amd import fem
    from tests.gpu_util import rel
    mesh, levels = make_pair(n0, r, 3, 0.1)
    lev = levels[-1]
    k = fem_inputs.k_exp_fourier(lev.vert_xyz)
    A = assemble.apply_bc(assemble.stiffness(lev, k), lev.boundary)
    b = _rhs(lev)
    u_ref = solvers.direct_solve(A, b, rtol=1e-14)
    S = fem.Solver(mesh, fem.SolveOptions(rtol=1e-10, precision=prec, smoother="patch")).setup(_t(k))
    u, res = S.solve(_t(b))
    Sj = fem.Solver(mesh, fem.SolveOptions(rtol=1e-10, precision=prec)).setup(_t(k))
    _, resj = Sj.solve(_t(b))
    torch.cuda.synchronize()
    print(f"iterations patch {res.iterations} jacobi {resj.iterations}", flush=True)
    assert res.rel_residual_true <= 1e-10
    assert rel(u.cpu().numpy(), u_ref) <= 1e-8
    assert res.iterations <= resj.iterations
    if prec == "fp64" and lev.n_dofs <= 400:
        pts = op.star_patches(lev)
        inv = op.patch_inverses(A, pts)
        Bd = np.stack([op.apply_patch_pc(pts, inv, lev.boundary, e) for e in np.eye(lev.n_dofs)], axis=1)
        lam = np.max(np.linalg.eigvals(Bd @ A.toarray()).real)
        est = res.lambda_max[len(levels) - 1]
        assert 0.9 * lam <= est <= lam * (1 + 1e-9)
