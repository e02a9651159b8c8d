"""torch.autograd wrappers: the PDE solve u(k, b) and the mass product, with hand-written
adjoints that run in the library's kernels.

Forward:  A_bc(k) u = b                    (multigrid-CG solve)
Backward: A_bc(k) lam = du_bar             (the same solve: A_bc is symmetric)
          dL/dk_v = - lam^T (dA/dk_v) u    (cell-wise grad(u).grad(lam) contraction with the P1
                                            hat function of vertex v, fem_adjoint_grad_k)
          dL/db   = lam
The gradient with respect to k is the Euclidean gradient with respect to its vertex values.
"""
from __future__ import annotations

import torch

from . import fem


class PoissonSolve(torch.autograd.Function):
    """u = PoissonSolve.apply(k, b, solver): k FP64 on the finest vertex lattice (or None for
    k = 1 when no gradient in k is needed), b FP64 on the finest dofs."""

    @staticmethod
    def forward(ctx, k, b, solver: "fem.Solver"):
        if k is not None and (solver.k is None or solver.k.data_ptr() != k.data_ptr()
                              or getattr(solver, "_k_version", None) != k._version):
            solver.setup(k.detach())
            solver._k_version = k._version
        u, res = solver.solve(b.detach().contiguous())
        ctx.solver = solver
        ctx.res = res
        ctx.save_for_backward(u)
        ctx.has_k = k is not None
        return u

    @staticmethod
    def backward(ctx, gu):
        (u,) = ctx.saved_tensors
        solver = ctx.solver
        lam, _ = solver.solve(gu.detach().contiguous())
        gk = solver.mesh.adjoint_grad_k(u, lam) if (ctx.has_k and ctx.needs_input_grad[0]) else None
        return gk, lam, None


class MassApply(torch.autograd.Function):
    """y = M x with the consistent mass matrix (symmetric, so the adjoint is M again)."""

    @staticmethod
    def forward(ctx, x, mesh: "fem.Mesh", level: int):
        ctx.mesh, ctx.level = mesh, level
        return mesh.mass(x.detach().contiguous(), level=level, bc="none")

    @staticmethod
    def backward(ctx, gy):
        return ctx.mesh.mass(gy.detach().contiguous(), level=ctx.level, bc="none"), None, None


def l2_misfit(u: torch.Tensor, u_obs: torch.Tensor, mesh: "fem.Mesh", level: int = -1) -> torch.Tensor:
    """J = 1/2 (u - u_obs)^T M (u - u_obs), the squared L2 norm of the misfit."""
    e = u - u_obs
    return 0.5 * torch.dot(e, MassApply.apply(e, mesh, level))
