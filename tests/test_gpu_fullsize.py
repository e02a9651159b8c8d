"""Parity at the benchmark sizes, in the launch configurations bench.py times.

* The actions bench.py times, on the finest level of the same hierarchies (the geometry from
  the coarsest level's table): P2 on 64^3 x 6 tetrahedra refined from 16^3, k = 1, FP64 against
  the oracle's matrix-free action to 1e-12, FP32 to 2e-6; P3 on 48^3 refined from 6^3 with
  k = exp(g), FP64 1e-12, FP32 2e-6; P2 on 128^3 refined from 4^3 (12.6M cells), FP64 1e-12; and
  P2 on a single-level 128^3 mesh (the geometry from the vertex coordinates), FP64 1e-12.
* The 128^3 x 6 action sweep on the hierarchy refined from 4^3: P1 (2.1M dofs) FP64 1e-12 /
  FP32 2e-6 against the oracle's full matrix-free action; P3 (57M dofs, the paper's own problem
  size) on sampled rows (seeded random dofs, dofs on brick planes, next to the boundary and on
  it) against the oracle's evaluation of those rows from the cells around them, FP64 1e-12 /
  FP32 2e-6 in the norm over the sample.
* The variable-coefficient P3 solve at full size (48^3, k = exp(g), f = 1, 4-level MG-CG, FP64 and
  mixed, rtol 1e-10) against sampled values of the oracle's solution (written by
  tests/golden/make_p3_48_vark_solution.py, oracle MG-CG to 1e-13): relative error over the
  sample and of the norm <= 1e-8.
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
@pytest.mark.parametrize("n0,refine,p,kvar", [(16, 2, 2, False), (6, 3, 3, True), (4, 5, 2, False),
                                              (128, 0, 2, False)])
def test_action_at_bench_size(n0, refine, p, kvar):
    n = n0 * 2 ** refine
    banner(f"full-size action n={n} (from {n0}^3) p={p} kvar={kvar}")
    from paper_2104_08012_amd import fem
    mesh = fem.Mesh(n0, refine, p, device="cuda:0")
    assert mesh.info(refine)["geometry"] == ("table" if refine >= 2 else "vertex")
    lev = om.single_level(n, p)   # the uniform refinement of the uniform n0^3 mesh is uniform
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


@pytest.mark.gpu
@pytest.mark.parametrize("p", [1, 3])
def test_action_sweep_128(p):
    banner(f"full-size action sweep n=128 p={p}")
    from paper_2104_08012_amd import fem
    n = 128
    mesh = fem.Mesh(4, 5, p, device="cuda:0")
    assert mesh.info(5)["geometry"] == "table"
    L = p * n + 1
    N = L ** 3
    lat = mesh.dof_lattice().astype(np.int64)
    perm = lat[:, 0] + L * (lat[:, 1] + L * lat[:, 2])     # library order -> oracle order
    x = fem_inputs.uniform_vector(N, 0)                   # oracle order
    x_lib = x[perm]
    y64 = mesh.apply(_t(x_lib)).cpu().numpy()
    y32 = mesh.apply(_t(x_lib, torch.float32)).double().cpu().numpy()
    torch.cuda.synchronize()
    del mesh
    torch.cuda.empty_cache()
    if p == 1:
        print("[fullsize] oracle P1 action ...", flush=True)
        lev = om.single_level(n, p)
        y_ref = assemble.matfree_action(lev, x, None)[perm]
        a64, a32 = y64, y32
    else:
        rng = np.random.default_rng(13)
        sample = rng.integers(0, N, 400).tolist()
        plane = rng.integers(0, L, (300, 3))
        plane[:100, 0] = rng.choice([12, 24, 192, 372, 373, 1, 2, L - 2], 100)
        plane[100:200, 1] = rng.choice([12, 13, 11, 96, 360], 100)
        plane[200:, 2] = rng.choice([0, 12, 24, L - 1, 372], 100)
        sample += [int(i + L * (j + L * k)) for i, j, k in plane]
        sample = np.unique(np.array(sample))
        print(f"[fullsize] oracle P3 action on {sample.size} sampled rows ...", flush=True)
        y_ref = assemble.action_at(n, p, om.uniform_vertices(n), x, sample)
        inv = np.empty(N, dtype=np.int64)
        inv[perm] = np.arange(N)                          # oracle index -> library index
        a64, a32 = y64[inv[sample]], y32[inv[sample]]
    e64, e32 = rel(a64, y_ref), rel(a32, y_ref)
    print(f"[fullsize] fp64 rel {e64:.2e}, fp32 rel {e32:.2e}", flush=True)
    assert e64 <= 1e-12
    assert e32 <= 2e-6


def _golden_p3():
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "p3_48_vark_solution.txt")
    head, idx, val = {}, [], []
    with open(path) as fh:
        for line in fh:
            if line.startswith("#"):
                continue
            a, b = line.split()
            if a.isdigit():
                idx.append(int(a))
                val.append(float(b))
            else:
                head[a] = float(b)
    return head, np.array(idx), np.array(val)


@pytest.mark.gpu
def test_p3_vark_solve_at_bench_size():
    banner("full-size solve P3 48^3 k=exp(g), 4 levels, fp64 and mixed, rtol 1e-10")
    from paper_2104_08012_amd import fem
    head, idx, u_ref = _golden_p3()
    mesh = fem.Mesh(6, 3, 3, device="cuda:0")
    L = 3 * 48 + 1
    lat = mesh.dof_lattice().astype(np.int64)
    perm = lat[:, 0] + L * (lat[:, 1] + L * lat[:, 2])
    inv = np.empty(L ** 3, dtype=np.int64)
    inv[perm] = np.arange(L ** 3)
    k = _t(fem_inputs.k_exp_fourier(mesh.vertex_coords()))
    b = mesh.mass(torch.ones(L ** 3, dtype=torch.float64, device="cuda:0"), bc="zero_rows")
    assert abs(torch.linalg.norm(b).item() - head["norm_b"]) <= 1e-12 * head["norm_b"]
    for prec in ("fp64", "mixed"):
        S = fem.Solver(mesh, fem.SolveOptions(rtol=1e-10, precision=prec)).setup(k)
        u, res = S.solve(b)
        torch.cuda.synchronize()
        nu = torch.linalg.norm(u).item()
        us = u.cpu().numpy()[inv[idx]]
        e = rel(us, u_ref)
        en = abs(nu - head["norm_u"]) / head["norm_u"]
        print(f"[fullsize] {prec}: {res.iterations} its, rel {res.rel_residual_true:.2e}, "
              f"sample err {e:.2e}, norm err {en:.2e}", flush=True)
        assert res.rel_residual_true <= 1e-10
        assert e <= 1e-8 and en <= 1e-8
        del S
