"""GPU checks of the adjoint gradient dJ/dk through torch.autograd.

* Against the oracle's gradient (direct FP64 solves) on a small jittered mesh: 1e-8.
* <g, k> = -lam^T b (A is linear in k).
* Central finite differences (step 1e-6, 20 directions, solves at rtol 1e-12) on the adjoint
  workload itself: P2 state on 32^3 x 6 tetrahedra from 8^3 refined twice, P1 coefficient,
  J = 1/2 ||u - u_obs||^2_{L2}, u_obs the solution for a seeded reference k plus 1 % noise,
  gradient at k = 1, f = 1.  Relative difference <= 1e-5 on every direction.
"""
import numpy as np
import pytest

import fem_inputs
from oracle import adjoint as oadj
from oracle import assemble
from tests.gpu_util import banner, make_pair, rel

torch = pytest.importorskip("torch")


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


@pytest.mark.gpu
@pytest.mark.parametrize("p", [1, 2, 3])
def test_gradient_matches_oracle(p):
    banner(f"adjoint vs oracle p={p}")
    from paper_2104_08012_amd import fem
    from paper_2104_08012_amd.autograd import PoissonSolve, l2_misfit
    mesh, levels = make_pair(2, 1, p, 0.1)
    lev = levels[-1]
    b = assemble.mass(lev) @ np.ones(lev.n_dofs)
    b[lev.boundary] = 0
    k_ref = fem_inputs.k_exp_fourier(lev.vert_xyz, seed=2)
    u_ref, _ = oadj.solve_state(lev, k_ref, b)
    u_obs = u_ref + 0.01 * np.max(np.abs(u_ref)) * fem_inputs.noise(lev.n_dofs)
    u_obs[lev.boundary] = 0
    k0 = fem_inputs.k_exp_fourier(lev.vert_xyz, seed=1)
    J_o, g_o, u_o, lam_o = oadj.gradient(lev, k0, b, u_obs)
    S = fem.Solver(mesh, fem.SolveOptions(rtol=1e-13, max_it=100))
    k = _t(k0).requires_grad_(True)
    bt = _t(b).requires_grad_(True)
    u = PoissonSolve.apply(k, bt, S)
    J = l2_misfit(u, _t(u_obs), mesh)
    J.backward()
    torch.cuda.synchronize()
    assert abs(J.item() - J_o) <= 1e-10 * abs(J_o)
    assert rel(k.grad.cpu().numpy(), g_o) <= 1e-8
    # dL/db = A_bc^-1 (M e): its boundary rows carry (M e)_B, which the oracle's adjoint
    # (right-hand side with boundary rows zeroed) leaves out; interior rows coincide.
    lam = bt.grad.cpu().numpy()
    I = lev.interior()
    assert rel(lam[I], lam_o[I]) <= 1e-8
    # linearity of A in k
    assert abs(k.grad.cpu().numpy() @ k0 + lam[I] @ b[I]) <= 1e-8 * abs(lam[I] @ b[I])


@pytest.mark.gpu
def test_finite_differences_adjoint_workload():
    banner("adjoint FD 32^3 P2")
    from paper_2104_08012_amd import fem
    from paper_2104_08012_amd.autograd import PoissonSolve, l2_misfit
    mesh = fem.Mesh(8, 2, 2, device="cuda:0")
    nv, n = mesh.n_vertices(), mesh.n_dofs()
    vxyz = mesh.vertex_coords()
    ones = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = mesh.mass(ones, bc="zero_rows")                      # f = 1
    S = fem.Solver(mesh, fem.SolveOptions(rtol=1e-12, max_it=100))
    k_ref = _t(fem_inputs.k_exp_fourier(vxyz, seed=2))
    u_ref = PoissonSolve.apply(k_ref, b, S)
    noise = _t(fem_inputs.noise(n))
    u_obs = u_ref + 0.01 * u_ref.abs().max() * noise
    lat = mesh.dof_lattice()
    L = 2 * 32
    bnd = _t(((lat == 0) | (lat == L)).any(axis=1).astype(np.float64))
    u_obs = u_obs * (1 - bnd)
    k0 = torch.ones(nv, dtype=torch.float64, device="cuda:0", requires_grad=True)
    J = l2_misfit(PoissonSolve.apply(k0, b, S), u_obs, mesh)
    J.backward()
    g = k0.grad.clone()

    def Jof(kk):
        with torch.no_grad():
            return l2_misfit(PoissonSolve.apply(kk, b, S), u_obs, mesh).item()

    eps = 1e-6
    worst = 0.0
    for d in fem_inputs.fd_directions(nv, 20):
        dt = _t(d)
        fd = (Jof(k0.detach() + eps * dt) - Jof(k0.detach() - eps * dt)) / (2 * eps)
        ad = torch.dot(g, dt).item()
        worst = max(worst, abs(fd - ad) / abs(ad))
    print(f"[fd] worst relative difference over 20 directions: {worst:.3e}", flush=True)
    assert worst <= 1e-5
