"""Lagrange P1-P3 on the reference tetrahedron, in exact rational arithmetic.

Follows the paper's FunctionSpace(mesh, "CG", degree) (Section 2, Listing 1):
continuous Lagrange elements with equispaced nodes.  The reference tetrahedron
has vertices (0,0,0), (1,0,0), (0,1,0), (0,0,1) and barycentric coordinates
l0 = 1-x-y-z, l1 = x, l2 = y, l3 = z.

Node order (local numbering used everywhere in the oracle):
  vertices 0..3;
  edge nodes, edges in the order (0,1),(0,2),(0,3),(1,2),(1,3),(2,3), the
  nodes of edge (a,b) ordered from vertex a towards vertex b;
  face nodes, faces in the order (0,1,2),(0,1,3),(0,2,3),(1,2,3).

Basis (Silvester's formula): phi_m = prod_i prod_{s<m_i} (p l_i - s)/(s+1),
m the barycentric multi-index of the node, |m| = p.

Monomial integral on the reference tetrahedron:
  int x^a y^b z^c = a! b! c! / (a+b+c+3)!.

Parity: pinned in tests/test_oracle_refelem.py against closed forms
(textbook P1 matrices, barycentric-monomial integration, integrals of the
basis) and invariants (symmetry, K.1 = 0, partition of unity, nodality).
"""
from __future__ import annotations

from fractions import Fraction
from functools import lru_cache
from itertools import product
from math import factorial

import numpy as np

EDGES = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))
FACES = ((0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3))

# A polynomial in (x, y, z) is a dict {(a, b, c): Fraction}.


def _padd(p, q):
    r = dict(p)
    for k, v in q.items():
        r[k] = r.get(k, Fraction(0)) + v
    return {k: v for k, v in r.items() if v != 0}


def _pmul(p, q):
    r = {}
    for (a1, b1, c1), v1 in p.items():
        for (a2, b2, c2), v2 in q.items():
            k = (a1 + a2, b1 + b2, c1 + c2)
            r[k] = r.get(k, Fraction(0)) + v1 * v2
    return {k: v for k, v in r.items() if v != 0}


def _pscale(p, s):
    return {k: v * s for k, v in p.items() if v * s != 0}


def _pderiv(p, d):
    r = {}
    for k, v in p.items():
        if k[d] == 0:
            continue
        kk = list(k)
        kk[d] -= 1
        r[tuple(kk)] = r.get(tuple(kk), Fraction(0)) + v * k[d]
    return {k: v for k, v in r.items() if v != 0}


def _peval(p, x, y, z):
    return sum(v * x ** a * y ** b * z ** c for (a, b, c), v in p.items())


def _bary(i):
    """Barycentric coordinate l_i as a polynomial."""
    if i == 0:
        return {(0, 0, 0): Fraction(1), (1, 0, 0): Fraction(-1),
                (0, 1, 0): Fraction(-1), (0, 0, 1): Fraction(-1)}
    e = [0, 0, 0]
    e[i - 1] = 1
    return {tuple(e): Fraction(1)}


def monomial_integral(a: int, b: int, c: int) -> Fraction:
    """int_T x^a y^b z^c dx over the reference tetrahedron."""
    return Fraction(factorial(a) * factorial(b) * factorial(c), factorial(a + b + c + 3))


def integrate(p) -> Fraction:
    return sum((v * monomial_integral(*k) for k, v in p.items()), Fraction(0))


@lru_cache(maxsize=None)
def node_multi_indices(p: int):
    """Barycentric multi-indices of the P_p nodes, in the local node order."""
    if p < 1 or p > 3:
        raise ValueError("degree must be 1, 2 or 3")
    nodes = []
    for v in range(4):
        m = [0, 0, 0, 0]
        m[v] = p
        nodes.append(tuple(m))
    for (a, b) in EDGES:
        for s in range(1, p):
            m = [0, 0, 0, 0]
            m[a] = p - s
            m[b] = s
            nodes.append(tuple(m))
    if p == 3:
        for (a, b, c) in FACES:
            m = [0, 0, 0, 0]
            m[a] = m[b] = m[c] = 1
            nodes.append(tuple(m))
    return tuple(nodes)


def nloc(p: int) -> int:
    return (p + 1) * (p + 2) * (p + 3) // 6


@lru_cache(maxsize=None)
def basis(p: int):
    """Silvester basis polynomials phi_m, in the local node order."""
    out = []
    lam = [_bary(i) for i in range(4)]
    for m in node_multi_indices(p):
        phi = {(0, 0, 0): Fraction(1)}
        for i in range(4):
            for s in range(m[i]):
                factor = _padd(_pscale(lam[i], Fraction(p, s + 1)),
                               {(0, 0, 0): Fraction(-s, s + 1)})
                phi = _pmul(phi, factor)
        out.append(phi)
    return tuple(out)


@lru_cache(maxsize=None)
def grad_basis(p: int):
    return tuple(tuple(_pderiv(phi, d) for d in range(3)) for phi in basis(p))


@lru_cache(maxsize=None)
def stiffness_tensors_exact(p: int):
    """S[a][b][i][j] = int d_a phi_i d_b phi_j (exact)."""
    g = grad_basis(p)
    n = nloc(p)
    return [[[[integrate(_pmul(g[i][a], g[j][b])) for j in range(n)] for i in range(n)]
             for b in range(3)] for a in range(3)]


@lru_cache(maxsize=None)
def weighted_stiffness_tensors_exact(p: int):
    """T[v][a][b][i][j] = int l_v d_a phi_i d_b phi_j (exact)."""
    g = grad_basis(p)
    n = nloc(p)
    lam = [_bary(i) for i in range(4)]
    return [[[[[integrate(_pmul(lam[v], _pmul(g[i][a], g[j][b]))) for j in range(n)]
               for i in range(n)] for b in range(3)] for a in range(3)] for v in range(4)]


@lru_cache(maxsize=None)
def mass_exact(p: int):
    phi = basis(p)
    n = nloc(p)
    return [[integrate(_pmul(phi[i], phi[j])) for j in range(n)] for i in range(n)]


@lru_cache(maxsize=None)
def basis_integrals_exact(p: int):
    return [integrate(phi) for phi in basis(p)]


def S(p: int) -> np.ndarray:
    """float64 array (3, 3, nloc, nloc)."""
    return np.array(stiffness_tensors_exact(p), dtype=np.float64)


def T(p: int) -> np.ndarray:
    """float64 array (4, 3, 3, nloc, nloc)."""
    return np.array(weighted_stiffness_tensors_exact(p), dtype=np.float64)


def M(p: int) -> np.ndarray:
    return np.array(mass_exact(p), dtype=np.float64)


def basis_integrals(p: int) -> np.ndarray:
    return np.array(basis_integrals_exact(p), dtype=np.float64)


def eval_basis(p: int, pts: np.ndarray) -> np.ndarray:
    """phi_i at reference points; pts (npts, 3) -> (npts, nloc) float64.

    Evaluated from the exact monomial coefficients.
    """
    pts = np.asarray(pts, dtype=np.float64).reshape(-1, 3)
    out = np.zeros((pts.shape[0], nloc(p)))
    for i, phi in enumerate(basis(p)):
        acc = np.zeros(pts.shape[0])
        for (a, b, c), v in phi.items():
            acc += float(v) * pts[:, 0] ** a * pts[:, 1] ** b * pts[:, 2] ** c
        out[:, i] = acc
    return out


def eval_basis_exact(p: int, x: Fraction, y: Fraction, z: Fraction):
    return [_peval(phi, x, y, z) for phi in basis(p)]


def reference_nodes(p: int):
    """Reference coordinates (x, y, z) of the nodes as exact fractions."""
    out = []
    for m in node_multi_indices(p):
        out.append((Fraction(m[1], p), Fraction(m[2], p), Fraction(m[3], p)))
    return out


def all_multi_indices(q: int):
    """All barycentric multi-indices with |m| = q (any order)."""
    return [m for m in product(range(q + 1), repeat=4) if sum(m) == q]
