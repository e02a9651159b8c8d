"""Parity at the benchmark sizes, in the launch configurations bench.py times.

* P2 on 64^3 x 6 tetrahedra, k = 1 (the default workload's finest level): the FP64 action
  against the oracle's matrix-free action to 1e-12, FP32 to 2e-6.
* P3 on 48^3 x 6 tetrahedra with k = exp(g): FP64 1e-12, FP32 2e-6.
* P2 on 128^3 x 6 tetrahedra (12.6M cells): FP64 1e-12.
* Solves at those sizes (seeded random right-hand side, boundary rows zero): the 3-level P2 64^3 MG-CG (FP64 and mixed, rtol 1e-10) and the P2
  128^3 MG-CG whose 32^3 coarse level is solved by nested MG-PCG (FP64 and mixed, rtol 1e-8).
  The oracle's FP64 action gives the residual ||b - A u|| / ||b|| of each returned solution,
  which must meet the requested tolerance.  FP64 and mixed solutions agree to 1e-8 at rtol
  1e-10; at rtol 1e-8 to 1e-6 (the residual tolerance times an allowance for the condition
  number).
"""
import numpy as np
import pytest

import fem_inputs
from oracle import assemble
from oracle import mesh as om
from tests.gpu_util import banner, rel

torch = pytest.importorskip("torch")


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda:0")


def _perm(mesh, lev):
    """Library dof order -> oracle (lexicographic lattice) order."""
    lat = mesh.dof_lattice().astype(np.int64)
    L = lev.n * lev.p + 1
    return lat[:, 0] + L * (lat[:, 1] + L * lat[:, 2])


def _oracle_residual(lev, k, b, u_lib, perm):
    u = np.empty(lev.n_dofs)
    u[perm] = u_lib
    r = b - assemble.matfree_action(lev, u, k)
    return np.linalg.norm(r) / np.linalg.norm(b)


@pytest.mark.gpu
@pytest.mark.parametrize("n,p,kvar", [(64, 2, False), (48, 3, True), (128, 2, False)])
def test_action_at_bench_size(n, p, kvar):
    banner(f"full-size action n={n} p={p} kvar={kvar}")
    from paper_2104_08012_amd import fem
    mesh = fem.Mesh(n, 0, p, device="cuda:0")
    lev = om.single_level(n, p)
    perm = _perm(mesh, lev)
    x = fem_inputs.uniform_vector(lev.n_dofs, 0)          # oracle order
    k = fem_inputs.k_exp_fourier(lev.vert_xyz) if kvar else None
    x_lib = x[perm]
    y64 = mesh.apply(_t(x_lib), _t(k) if kvar else None).cpu().numpy()
    y32 = None
    if n <= 64:
        y32 = mesh.apply(_t(x_lib, torch.float32), _t(k, torch.float32) if kvar else None).cpu().numpy()
    torch.cuda.synchronize()
    print("[fullsize] GPU done, oracle action ...", flush=True)
    y_ref = assemble.matfree_action(lev, x, k)[perm]
    e64 = rel(y64, y_ref)
    print(f"[fullsize] fp64 rel {e64:.2e}", flush=True)
    assert e64 <= 1e-12
    if y32 is not None:
        e32 = rel(y32, y_ref)
        print(f"[fullsize] fp32 rel {e32:.2e}", flush=True)
        assert e32 <= 2e-6


@pytest.mark.gpu
@pytest.mark.parametrize("n0,refine,used,rtol", [(16, 2, 0, 1e-10), (4, 5, 3, 1e-8)])
def test_solve_at_bench_size(n0, refine, used, rtol):
    banner(f"full-size solve n0={n0} refine={refine} used={used} rtol={rtol}")
    from paper_2104_08012_amd import fem
    n = n0 * 2 ** refine
    lev = om.single_level(n, 2)
    b = fem_inputs.uniform_vector(lev.n_dofs, 8)          # oracle order, boundary rows zero
    b[lev.boundary] = 0.0
    mesh = fem.Mesh(n0, refine, 2, device="cuda:0")
    perm = _perm(mesh, lev)
    bt = _t(b[perm])
    sols = {}
    for prec in ("fp64", "mixed"):
        S = fem.Solver(mesh, fem.SolveOptions(rtol=rtol, precision=prec, n_levels_used=used)).setup()
        u, res = S.solve(bt)
        torch.cuda.synchronize()
        print(f"[fullsize] {prec}: {res.iterations} its, coarse its {res.coarse_iterations}, "
              f"rel {res.rel_residual_true:.2e}", flush=True)
        assert res.rel_residual_true <= rtol
        if used:
            assert res.coarse_iterations > 0
        sols[prec] = u.cpu().numpy()
        del S
    del mesh, bt
    torch.cuda.empty_cache()
    print("[fullsize] oracle residuals ...", flush=True)
    for prec, u in sols.items():
        r = _oracle_residual(lev, None, b, u, perm)
        print(f"[fullsize] oracle residual {prec}: {r:.2e}", flush=True)
        assert r <= 1.01 * rtol
    d = rel(sols["mixed"], sols["fp64"])
    print(f"[fullsize] mixed vs fp64: {d:.2e}", flush=True)
    assert d <= (1e-8 if rtol <= 1e-10 else 1e-6)
