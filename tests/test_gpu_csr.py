"""GPU parity of the assembled operator (CSR values and SpMV) against the oracle's assembled
matrix A_bc = P_I A P_I + P_B, through the C ABI.

* Values (k = 1 and P1 k, uniform and jittered meshes, P1-P3): max |A - A_ref| <= 1e-13 max |A_ref|
  (element matrices by the same quadrature rule, summed in a different order).
* SpMV in FP64 vs the oracle's matrix product and vs the library's matrix-free action: 1e-12;
  FP32 values and vectors: 2e-6.  Repeated products are bitwise equal.
"""
import numpy as np
import pytest

import fem_inputs
from tests.gpu_util import banner, make_pair, oracle_A, rel

torch = pytest.importorskip("torch")


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda:0")


@pytest.mark.gpu
@pytest.mark.parametrize("n,p,jit,kvar", [(4, 1, 0.15, True), (4, 2, 0.0, False), (4, 2, 0.15, True),
                                          (2, 3, 0.1, True), (5, 2, 0.0, True)])
def test_csr_values_and_spmv(n, p, jit, kvar):
    banner(f"csr n={n} p={p} jit={jit} kvar={kvar}")
    import scipy.sparse as sp
    from paper_2104_08012_amd import fem
    mesh, levels = make_pair(n, 0, p, jit)
    lev = levels[0]
    k = fem_inputs.k_exp_fourier(lev.vert_xyz) if kvar else None
    A = fem.CsrOperator(mesh, 0)
    rp, col = A.pattern()
    vals = A.assemble(_t(k) if kvar else None)
    torch.cuda.synchronize()
    Ag = sp.csr_matrix((vals.cpu().numpy(), col, rp), shape=(A.n_rows, A.n_rows))
    Ar = oracle_A(lev, k)
    assert abs(Ag - Ar).max() <= 1e-13 * abs(Ar).max()
    x = fem_inputs.uniform_vector(lev.n_dofs, 0)
    y = A.spmv(vals, _t(x))
    y2 = A.spmv(vals, _t(x))
    ymf = mesh.apply(_t(x), _t(k) if kvar else None, level=0)
    torch.cuda.synchronize()
    assert rel(y.cpu().numpy(), Ar @ x) <= 1e-12
    assert rel(y.cpu().numpy(), ymf.cpu().numpy()) <= 1e-12
    assert torch.equal(y, y2)
    v32 = A.assemble(_t(k) if kvar else None, dtype=torch.float32)
    y32 = A.spmv(v32, _t(x, torch.float32))
    torch.cuda.synchronize()
    assert rel(y32.cpu().numpy(), Ar @ x) <= 2e-6
