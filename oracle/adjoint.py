"""Gradient of J(k) = 1/2 ||u(k) - u_obs||^2_{L2} with respect to the vertex
values of a P1 coefficient k, by the adjoint method.

The paper motivates sensitivities of simulations to their inputs (Section 1:
users need to compute sensitivities and optimise parameters); the operator is
the weak form of Section 2, eq. (4) with a coefficient k.

Definitions (all FP64):
  A_bc(k) u = b                        (state; A linear in k)
  J = 1/2 e^T M e,  e = u - u_obs      (M the consistent mass matrix)
  A_bc(k) lam = P_I M e                (adjoint; A_bc is symmetric)
  dJ/dk_v = -lam^T (dA/dk_v) u = - sum_K lam_K^T (sum_ab G_ab T^{v,ab}) u_K

Reading: the gradient is the Euclidean (nodal) gradient with respect to the
vertex values, which is what central differences on nodal perturbations
measure.

Parity: pinned by <g, k> = -lam^T b (A is linear in k), central differences
and a Taylor remainder test, in tests/test_oracle_adjoint.py.
"""
from __future__ import annotations

import numpy as np

from . import assemble, refelem
from .mesh import Level


def gradient_from_fields(level: Level, u: np.ndarray, lam: np.ndarray, k_vertex=None) -> np.ndarray:
    """g_v = - sum_K lam_K^T (sum_ab G_ab T^{v,ab}) u_K  (k_vertex is unused:
    A depends linearly on k, so dA/dk_v does not involve k)."""
    G, _ = level.geometric_factors()
    Tt = refelem.T(level.p)                                   # (4, 3, 3, nl, nl)
    uK = u[level.cell_dofs]
    lK = lam[level.cell_dofs]
    # per cell and vertex: sum_ab G_ab lam^T T^{v,ab} u
    gK = -np.einsum("cab,vabij,ci,cj->cv", G, Tt, lK, uK)
    return np.bincount(level.cell_vert.ravel(), weights=gK.ravel(), minlength=level.n_vertices)


def objective(level: Level, u: np.ndarray, u_obs: np.ndarray, Mmat=None) -> float:
    Mmat = assemble.mass(level) if Mmat is None else Mmat
    e = u - u_obs
    return 0.5 * float(e @ (Mmat @ e))


def solve_state(level: Level, k_vertex, b):
    from .solvers import direct_solve
    A = assemble.apply_bc(assemble.stiffness(level, k_vertex), level.boundary)
    return direct_solve(A, b), A


def gradient(level: Level, k_vertex, b, u_obs):
    """Returns (J, g, u, lam) with direct FP64 solves."""
    from .solvers import direct_solve
    u, A = solve_state(level, k_vertex, b)
    Mmat = assemble.mass(level)
    e = u - u_obs
    rhs = Mmat @ e
    rhs[level.boundary] = 0.0
    lam = direct_solve(A, rhs)
    g = gradient_from_fields(level, u, lam)
    return 0.5 * float(e @ (Mmat @ e)), g, u, lam
