"""The allocation-free operator action, fem_apply_laplacian_noalloc, against fem_apply_laplacian,
through the C ABI.

Both run the same kernels; the allocation-free entry point keeps the interface partial sums in
the library's file-scope device array instead of the mesh buffer.  Its results must equal the
existing entry point's bit for bit (the parity bar of the action is 1e-12 relative in FP64 and
2e-6 in FP32; equality is stronger) on two calls in a row, the second on a smaller level, for
P1-P3, FP64 and FP32, k = 1 and a P1 coefficient, all boundary-row modes.  A level whose partial
sums exceed the array is refused before anything is enqueued.
"""
import numpy as np
import pytest

import fem_inputs
from tests.gpu_util import banner

torch = pytest.importorskip("torch")


def _call(name, mesh, level, x, k, y, flags):
    from paper_2104_08012_amd import _lib as L
    dt = L.FEM_F64 if x.dtype == torch.float64 else L.FEM_F32
    kp = None if k is None else k.data_ptr()
    return getattr(L.lib(), name)(mesh.handle, level, dt, kp, x.data_ptr(), y.data_ptr(), flags,
                                  torch.cuda.current_stream().cuda_stream)


@pytest.mark.gpu
@pytest.mark.parametrize("p", [1, 2, 3])
def test_noalloc_action_equals_action(p):
    banner(f"noalloc action p={p}")
    from paper_2104_08012_amd import fem
    from paper_2104_08012_amd import _lib as L
    mesh = fem.Mesh(4, 2, p, jitter=fem_inputs.jitter_offsets(4, 0.1), device="cuda:0")
    for level in (2, 1):                      # 16^3 cubes, then the smaller 8^3 level
        n = mesh.n_dofs(level)
        kv = torch.as_tensor(fem_inputs.k_exp_fourier(mesh.vertex_coords(level)), device="cuda:0")
        for dtype in (torch.float64, torch.float32):
            x = torch.as_tensor(fem_inputs.uniform_vector(n, level), device="cuda:0").to(dtype)
            for k in (None, kv.to(dtype)):
                for flags in (L.FEM_BC_IDENTITY, L.FEM_BC_NONE, L.FEM_BC_ZERO_ROWS):
                    y_ref = torch.full_like(x, float("nan"))
                    y = torch.full_like(x, float("nan"))
                    assert _call("fem_apply_laplacian", mesh, level, x, k, y_ref, flags) == L.FEM_OK
                    assert _call("fem_apply_laplacian_noalloc", mesh, level, x, k, y, flags) == L.FEM_OK
                    torch.cuda.synchronize()
                    assert torch.isfinite(y).all()
                    assert torch.equal(y, y_ref), (level, dtype, k is None, flags)


@pytest.mark.gpu
def test_noalloc_action_refuses_oversized_level():
    banner("noalloc action oversized level")
    from paper_2104_08012_amd import fem
    from paper_2104_08012_amd import _lib as L
    mesh = fem.Mesh(64, 0, 3, device="cuda:0")     # P3 64^3: 8 x 1.74M interface slots, 111 MB
    n = mesh.n_dofs(0)
    x = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    y = torch.full_like(x, 7.0)
    assert _call("fem_apply_laplacian_noalloc", mesh, 0, x, None, y, L.FEM_BC_IDENTITY) == L.FEM_ERR_WORKSPACE
    torch.cuda.synchronize()
    assert float(y.min()) == 7.0 and float(y.max()) == 7.0        # nothing was enqueued
