"""MI355X (gfx950) matrix-free Lagrange P1-P3 Poisson operator, multigrid-preconditioned CG and
adjoint coefficient gradient, behind a C ABI (include/fem.h).

Importing the package loads nothing; the HIP library is loaded on first use and must have been
built in-tree (there is no CPU fallback).
"""
__all__ = ["Mesh", "Solver", "SolveOptions", "PatchPreconditioner", "CsrOperator", "PoissonSolve"]


def __getattr__(name):
    if name in ("Mesh", "Solver", "SolveOptions", "PatchPreconditioner", "CsrOperator"):
        from . import fem
        return getattr(fem, name)
    if name == "PoissonSolve":
        from .autograd import PoissonSolve
        return PoissonSolve
    raise AttributeError(name)
