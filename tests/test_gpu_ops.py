"""GPU parity of the cell-wise kernels against the oracle, through the C ABI.

Tolerances: FP64 actions 1e-12 relative (2-norm, random x ~ U(-1,1)); FP32 actions 2e-6
relative (single-precision rounding of ~30 terms per entry on the uniform mesh); transfers,
diagonal, mass and gradient 1e-12 in FP64.  Mesh sizes span several bricks and odd sizes that
fall back to smaller bricks (n = 5: 1-cube bricks, n = 6: 2-cube bricks); for P2 the cube kernel
merges R bricks along x per workgroup: n = 16 (4 bricks per direction) R = 4, n = 8 R = 2,
n = 12 (3 bricks) R = 1.
"""
import numpy as np
import pytest

import fem_inputs
from oracle import adjoint as oadj
from oracle import assemble, transfer
from tests.gpu_util import banner, make_pair, oracle_A, rel

torch = pytest.importorskip("torch")

CASES = [(5, 1, 0.0), (6, 2, 0.15), (8, 1, 0.0), (8, 2, 0.15), (8, 3, 0.15), (12, 2, 0.0), (16, 2, 0.15),
         (4, 3, 0.0)]


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda:0")


@pytest.mark.gpu
@pytest.mark.parametrize("n,p,jit", CASES)
@pytest.mark.parametrize("kvar", [False, True])
def test_apply_fp64_parity(n, p, jit, kvar):
    banner(f"apply fp64 n={n} p={p} jit={jit} kvar={kvar}")
    mesh, levels = make_pair(n, 0, p, jit)
    lev = levels[0]
    k = fem_inputs.k_exp_fourier(lev.vert_xyz) if kvar else None
    x = fem_inputs.uniform_vector(lev.n_dofs, 0)
    kt = _t(k) if kvar else None
    for bc in ("identity", "none", "zero_rows"):
        y = mesh.apply(_t(x), kt, level=0, bc=bc)
        torch.cuda.synchronize()
        y_ref = oracle_A(lev, k, bc) @ x
        assert rel(y.cpu().numpy(), y_ref) <= 1e-12, bc


@pytest.mark.gpu
@pytest.mark.parametrize("n,p,jit", [(8, 2, 0.15), (16, 2, 0.15), (6, 3, 0.0), (5, 1, 0.15), (8, 1, 0.15)])
@pytest.mark.parametrize("kvar", [False, True])
def test_apply_fp32_parity(n, p, jit, kvar):
    banner(f"apply fp32 n={n} p={p} kvar={kvar}")
    mesh, levels = make_pair(n, 0, p, jit)
    lev = levels[0]
    k = fem_inputs.k_exp_fourier(lev.vert_xyz) if kvar else None
    x = fem_inputs.uniform_vector(lev.n_dofs, 0)
    y = mesh.apply(_t(x, torch.float32), _t(k, torch.float32) if kvar else None, level=0)
    torch.cuda.synchronize()
    y_ref = oracle_A(lev, k) @ x
    assert rel(y.cpu().numpy(), y_ref) <= 2e-6


@pytest.mark.gpu
@pytest.mark.parametrize("n,r,p,jit", [(2, 3, 1, 0.15), (2, 3, 2, 0.15), (3, 2, 2, 0.15), (1, 4, 2, 0.0),
                                       (2, 2, 3, 0.15), (3, 2, 3, 0.15)])
@pytest.mark.parametrize("kvar", [False, True])
def test_apply_refined_levels_parity(n, r, p, jit, kvar):
    """Every level of a refined hierarchy: from level 2 on, a 4-cube brick lies inside one cube of
    the coarsest level and the action takes the geometry from the coarsest level's table (P1/P2:
    the cube kernel, in place of the vertex coordinates; P3: the lattice kernel, in place of the
    per-cell factors).  n = 2 -> 16: R = 2 and 4 bricks per workgroup; n = 3 -> 12: R = 1, a
    coarsest level of odd size; n = 1 -> 16: a single coarsest cube."""
    banner(f"apply refined n={n} r={r} p={p} jit={jit} kvar={kvar}")
    mesh, levels = make_pair(n, r, p, jit)
    for ell, lev in enumerate(levels):
        k = fem_inputs.k_exp_fourier(lev.vert_xyz) if kvar else None
        x = fem_inputs.uniform_vector(lev.n_dofs, ell)
        y_ref = oracle_A(lev, k) @ x
        y = mesh.apply(_t(x), _t(k) if kvar else None, level=ell)
        y32 = mesh.apply(_t(x, torch.float32), _t(k, torch.float32) if kvar else None, level=ell)
        torch.cuda.synchronize()
        assert rel(y.cpu().numpy(), y_ref) <= 1e-12, ell
        assert rel(y32.cpu().numpy(), y_ref) <= 2e-6, ell


@pytest.mark.gpu
@pytest.mark.parametrize("n", [8, 16])
def test_apply_axpby_and_determinism(n):
    banner(f"apply axpby / determinism n={n}")
    mesh, levels = make_pair(n, 0, 2, 0.15)
    lev = levels[0]
    x = fem_inputs.uniform_vector(lev.n_dofs, 0)
    z = fem_inputs.uniform_vector(lev.n_dofs, 7)
    xt, zt = _t(x), _t(z)
    y1 = mesh.apply(xt)
    y2 = mesh.apply(xt)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)
    r = zt.clone()
    mesh.apply(xt, out=r, alpha=-1.0, z=r, beta=1.0)      # in place: r = z - A x
    torch.cuda.synchronize()
    ref = z - oracle_A(lev) @ x
    assert rel(r.cpu().numpy(), ref) <= 1e-12


@pytest.mark.gpu
@pytest.mark.parametrize("n,p,dtype", [(32, 2, "f64"), (32, 2, "f32"), (24, 2, "f64"), (32, 1, "f64"),
                                       (64, 2, "f64")])
def test_apply_repeated_launches_bitwise(n, p, dtype):
    """Back-to-back actions on alternating inputs share the level's interface slots: 40 launches
    without synchronisation (and the in-place axpby form y = z - A x) must each equal the first
    launch on the same input bit for bit, and that one the oracle."""
    banner(f"repeated launches n={n} p={p} {dtype}")
    dt = torch.float64 if dtype == "f64" else torch.float32
    mesh, levels = make_pair(n, 0, p, 0.1 if n <= 32 else 0.0)
    lev = levels[0]
    xs = [_t(fem_inputs.uniform_vector(lev.n_dofs, s), dt) for s in (0, 1)]
    ref = [mesh.apply(x) for x in xs]
    torch.cuda.synchronize()
    if n <= 32:
        y0 = oracle_A(lev) @ fem_inputs.uniform_vector(lev.n_dofs, 0)
        assert rel(ref[0].double().cpu().numpy(), y0) <= (1e-12 if dtype == "f64" else 2e-6)
    outs = [torch.empty_like(xs[0]) for _ in range(40)]
    for i, y in enumerate(outs):
        mesh.apply(xs[i % 2], out=y)
    zs = [x.clone() for x in xs]
    for i in range(10):                      # r = z - A x in place, alternating inputs
        zs[i % 2].copy_(xs[(i + 1) % 2])
        mesh.apply(xs[i % 2], out=zs[i % 2], alpha=-1.0, z=zs[i % 2], beta=1.0)
        torch.cuda.synchronize()
        assert torch.equal(zs[i % 2], xs[(i + 1) % 2] - ref[i % 2]), i
    torch.cuda.synchronize()
    for i, y in enumerate(outs):
        assert torch.equal(y, ref[i % 2]), i


@pytest.mark.gpu
@pytest.mark.parametrize("n,p,jit", [(8, 2, 0.15), (6, 3, 0.0), (5, 1, 0.0)])
def test_mass_parity(n, p, jit):
    banner(f"mass n={n} p={p}")
    mesh, levels = make_pair(n, 0, p, jit)
    lev = levels[0]
    x = fem_inputs.uniform_vector(lev.n_dofs, 0)
    M = assemble.mass(lev)
    y = mesh.mass(_t(x), level=0, bc="none")
    yz = mesh.mass(_t(x), level=0, bc="zero_rows")
    torch.cuda.synchronize()
    assert rel(y.cpu().numpy(), M @ x) <= 1e-12
    ref = M @ x
    ref[lev.boundary] = 0
    assert rel(yz.cpu().numpy(), ref) <= 1e-12


@pytest.mark.gpu
@pytest.mark.parametrize("n,p,jit", [(8, 2, 0.15), (6, 3, 0.0), (5, 1, 0.0)])
@pytest.mark.parametrize("kvar", [False, True])
def test_diagonal_parity(n, p, jit, kvar):
    banner(f"diag n={n} p={p} kvar={kvar}")
    mesh, levels = make_pair(n, 0, p, jit)
    lev = levels[0]
    k = fem_inputs.k_exp_fourier(lev.vert_xyz) if kvar else None
    d = mesh.diagonal(_t(k) if kvar else None, level=0)
    torch.cuda.synchronize()
    assert rel(d.cpu().numpy(), oracle_A(lev, k).diagonal()) <= 1e-12


@pytest.mark.gpu
@pytest.mark.parametrize("n,p,jit", [(2, 1, 0.0), (4, 2, 0.15), (3, 3, 0.15), (6, 2, 0.0), (4, 3, 0.0)])
def test_transfer_parity(n, p, jit):
    banner(f"transfers n={n} p={p}")
    mesh, levels = make_pair(n, 1, p, jit)
    P = transfer.prolongation(levels[0], levels[1])
    xc = fem_inputs.uniform_vector(levels[0].n_dofs, 0)
    xf0 = fem_inputs.uniform_vector(levels[1].n_dofs, 1)
    xf = _t(xf0)
    mesh.prolong(_t(xc), xf, 1)
    rf = fem_inputs.uniform_vector(levels[1].n_dofs, 2)
    rc = mesh.restrict(_t(rf), 1)
    torch.cuda.synchronize()
    assert rel(xf.cpu().numpy(), xf0 + P @ xc) <= 1e-12
    rc_ref = P.T @ rf
    rc_ref[levels[0].boundary] = 0
    assert rel(rc.cpu().numpy(), rc_ref) <= 1e-12
    xf32 = _t(xf0, torch.float32)
    mesh.prolong(_t(xc, torch.float32), xf32, 1)
    rc32 = mesh.restrict(_t(rf, torch.float32), 1)
    torch.cuda.synchronize()
    assert rel(xf32.cpu().numpy(), xf0 + P @ xc) <= 2e-6
    assert rel(rc32.cpu().numpy(), rc_ref) <= 2e-6


@pytest.mark.gpu
@pytest.mark.parametrize("p", [1, 2])
def test_transfer_parity_large_levels(p):
    """32^3 -> 64^3: from 32 coarse cubes per direction P1/P2 prolong one thread per coarse cube
    (compile-time weights) instead of one thread per fine dof; the restriction runs the
    compile-time class stencils at every size."""
    banner(f"transfers 32^3 -> 64^3 p={p}")
    mesh, levels = make_pair(32, 1, p, 0.0)
    P = transfer.prolongation(levels[0], levels[1])
    xc = fem_inputs.uniform_vector(levels[0].n_dofs, 0)
    xf0 = fem_inputs.uniform_vector(levels[1].n_dofs, 1)
    rf = fem_inputs.uniform_vector(levels[1].n_dofs, 2)
    rc_ref = P.T @ rf
    rc_ref[levels[0].boundary] = 0
    for dt, tol in ((torch.float64, 1e-12), (torch.float32, 2e-6)):
        xf = _t(xf0, dt)
        mesh.prolong(_t(xc, dt), xf, 1)
        rc = mesh.restrict(_t(rf, dt), 1)
        torch.cuda.synchronize()
        assert rel(xf.double().cpu().numpy(), xf0 + P @ xc) <= tol, dt
        assert rel(rc.double().cpu().numpy(), rc_ref) <= tol, dt


@pytest.mark.gpu
@pytest.mark.parametrize("n,p,jit", [(8, 2, 0.15), (6, 3, 0.0), (5, 1, 0.15), (4, 2, 0.0)])
def test_adjoint_grad_parity(n, p, jit):
    banner(f"grad n={n} p={p}")
    mesh, levels = make_pair(n, 0, p, jit)
    lev = levels[0]
    u = fem_inputs.uniform_vector(lev.n_dofs, 0)
    lam = fem_inputs.uniform_vector(lev.n_dofs, 1)
    u[lev.boundary] = 0
    lam[lev.boundary] = 0
    g = mesh.adjoint_grad_k(_t(u), _t(lam), level=0)
    torch.cuda.synchronize()
    g_ref = oadj.gradient_from_fields(lev, u, lam)
    assert rel(g.cpu().numpy(), g_ref) <= 1e-12


@pytest.mark.gpu
def test_invalid_arguments_rejected_before_launch():
    from paper_2104_08012_amd._lib import FemError
    mesh, levels = make_pair(4, 0, 2, 0.0)
    x = torch.zeros(levels[0].n_dofs, dtype=torch.float64, device="cuda:0")
    with pytest.raises(ValueError):
        mesh.apply(x[:-1])
    with pytest.raises(FemError):
        mesh.apply(x, out=x)
    with pytest.raises(FemError):
        mesh.info(7)
