"""Conical-product (collapsed Gauss-Jacobi) quadrature on the reference tetrahedron.

Stroud's construction: map the unit cube to the tetrahedron by
  x = u, y = v (1-u), z = w (1-u)(1-v)
with Jacobian (1-u)^2 (1-v); integrate u with Gauss-Jacobi(alpha=2), v with
Gauss-Jacobi(alpha=1) and w with Gauss-Legendre, all shifted to [0, 1].  With m
points per direction the rule is exact for total degree 2m-1.

Used only for load vectors and L2 errors of manufactured solutions (the
paper's error check, Section 2 after eq. 3).

Parity: pinned against the closed-form monomial integrals in
tests/test_oracle_refelem.py.
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np
from scipy.special import roots_jacobi


def _gj01(m: int, alpha: float):
    """Gauss-Jacobi nodes/weights for int_0^1 (1-t)^alpha g(t) dt."""
    x, w = roots_jacobi(m, alpha, 0.0)          # weight (1-x)^alpha on [-1, 1]
    t = 0.5 * (x + 1.0)
    return t, w * 0.5 ** (alpha + 1.0)


@lru_cache(maxsize=None)
def conical_product_rule(degree: int):
    """(points (nq, 3), weights (nq,)) exact for polynomials of total degree <= degree."""
    m = max(1, (degree + 2) // 2)
    u, wu = _gj01(m, 2.0)
    v, wv = _gj01(m, 1.0)
    w, ww = _gj01(m, 0.0)
    U, V, W = np.meshgrid(u, v, w, indexing="ij")
    WU, WV, WW = np.meshgrid(wu, wv, ww, indexing="ij")
    x = U
    y = V * (1.0 - U)
    z = W * (1.0 - U) * (1.0 - V)
    pts = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    wts = (WU * WV * WW).ravel()
    return pts, wts
