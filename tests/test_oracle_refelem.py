"""Pins for the oracle's reference element (exact rationals).

Independent routes used here:
* gradients of barycentric coordinates are constant vectors, which gives the
  P1 stiffness matrix in closed form;
* integrals of barycentric monomials on a simplex,
      int_T l0^a l1^b l2^c l3^d = a! b! c! d! 3! |T| / (a+b+c+d+3)!,
  give mass matrices and basis integrals by a route that never expands
  anything in x, y, z (the oracle integrates monomials in x, y, z);
* invariants: symmetry, row sums, kernel, partition of unity, nodality.
"""
from fractions import Fraction
from itertools import product
from math import factorial

import numpy as np
import pytest

from oracle import quadrature, refelem

VOL = Fraction(1, 6)
GRAD_LAMBDA = [(-1, -1, -1), (1, 0, 0), (0, 1, 0), (0, 0, 1)]


# --- barycentric-polynomial algebra (independent of the oracle's xyz route) ---

def _bmul(p, q):
    r = {}
    for k1, v1 in p.items():
        for k2, v2 in q.items():
            k = tuple(a + b for a, b in zip(k1, k2))
            r[k] = r.get(k, Fraction(0)) + v1 * v2
    return r


def _bint(p):
    out = Fraction(0)
    for (a, b, c, d), v in p.items():
        out += v * Fraction(factorial(a) * factorial(b) * factorial(c) * factorial(d) * 6,
                            factorial(a + b + c + d + 3)) * VOL
    return out


def _bderiv(p, i):
    r = {}
    for k, v in p.items():
        if k[i]:
            kk = list(k)
            kk[i] -= 1
            r[tuple(kk)] = r.get(tuple(kk), Fraction(0)) + v * k[i]
    return r


def _silvester_bary(p, m):
    phi = {(0, 0, 0, 0): Fraction(1)}
    for i in range(4):
        for s in range(m[i]):
            e = [0, 0, 0, 0]
            e[i] = 1
            phi = _bmul(phi, {tuple(e): Fraction(p, s + 1), (0, 0, 0, 0): Fraction(-s, s + 1)})
    return phi


def _bary_mass(p):
    phis = [_silvester_bary(p, m) for m in refelem.node_multi_indices(p)]
    return [[_bint(_bmul(a, b)) for b in phis] for a in phis]


def _bary_stiffness(p):
    phis = [_silvester_bary(p, m) for m in refelem.node_multi_indices(p)]
    d = [[_bderiv(phi, i) for i in range(4)] for phi in phis]
    n = len(phis)
    S = [[[[Fraction(0)] * n for _ in range(n)] for _ in range(3)] for _ in range(3)]
    for j, k in product(range(n), repeat=2):
        for i, l in product(range(4), repeat=2):
            val = _bint(_bmul(d[j][i], d[k][l]))
            if val == 0:
                continue
            for a, b in product(range(3), repeat=2):
                S[a][b][j][k] += GRAD_LAMBDA[i][a] * GRAD_LAMBDA[l][b] * val
    return S


# --- node order convention (local numbering) ---

def test_node_order_convention():
    assert refelem.node_multi_indices(1) == ((1, 0, 0, 0), (0, 1, 0, 0), (0, 0, 1, 0), (0, 0, 0, 1))
    assert refelem.node_multi_indices(2)[4:] == (
        (1, 1, 0, 0), (1, 0, 1, 0), (1, 0, 0, 1), (0, 1, 1, 0), (0, 1, 0, 1), (0, 0, 1, 1))
    p3 = refelem.node_multi_indices(3)
    assert p3[4:6] == ((2, 1, 0, 0), (1, 2, 0, 0))          # edge 01, near vertex 0 first
    assert p3[14:16] == ((0, 0, 2, 1), (0, 0, 1, 2))        # edge 23
    assert p3[16:] == ((1, 1, 1, 0), (1, 1, 0, 1), (1, 0, 1, 1), (0, 1, 1, 1))
    for p in (1, 2, 3):
        assert len(refelem.node_multi_indices(p)) == refelem.nloc(p) == (p + 1) * (p + 2) * (p + 3) // 6


def test_p1_stiffness_closed_form():
    # K_ij = |T| grad(l_i) . grad(l_j) with constant barycentric gradients
    S = refelem.stiffness_tensors_exact(1)
    K = [[sum(S[a][a][i][j] for a in range(3)) for j in range(4)] for i in range(4)]
    expect = [[VOL * sum(GRAD_LAMBDA[i][a] * GRAD_LAMBDA[j][a] for a in range(3)) for j in range(4)]
              for i in range(4)]
    assert K == expect
    assert K[0] == [Fraction(1, 2), Fraction(-1, 6), Fraction(-1, 6), Fraction(-1, 6)]


def test_p1_mass_and_integrals_closed_form():
    M = refelem.mass_exact(1)
    for i, j in product(range(4), repeat=2):
        assert M[i][j] == (Fraction(1, 60) if i == j else Fraction(1, 120))
    assert refelem.basis_integrals_exact(1) == [Fraction(1, 24)] * 4


@pytest.mark.parametrize("p", [1, 2, 3])
def test_mass_matches_barycentric_route(p):
    assert refelem.mass_exact(p) == _bary_mass(p)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_stiffness_matches_barycentric_route(p):
    assert refelem.stiffness_tensors_exact(p) == _bary_stiffness(p)


def test_p2_textbook_mass_entries():
    # quadratic tetrahedron mass matrix in units of |T|/420
    M = refelem.mass_exact(2)
    u = VOL / 420
    assert M[0][0] == 6 * u and M[0][1] == 1 * u
    assert M[0][4] == -4 * u      # vertex 0 with edge 01
    assert M[0][7] == -6 * u      # vertex 0 with edge 12 (opposite)
    assert M[4][4] == 32 * u
    assert M[4][5] == 16 * u      # edges 01 and 02 share vertex 0
    assert M[4][9] == 8 * u       # edges 01 and 23 are opposite


def test_basis_integrals_closed_form():
    # int phi over |T| = 1/6: P2 vertex -|T|/20, edge |T|/5; P3 vertex |T|/40, edge 0, face 9|T|/40
    b2 = refelem.basis_integrals_exact(2)
    assert b2[:4] == [Fraction(-1, 120)] * 4 and b2[4:] == [Fraction(1, 30)] * 6
    b3 = refelem.basis_integrals_exact(3)
    assert b3[:4] == [Fraction(1, 240)] * 4
    assert b3[4:16] == [Fraction(0)] * 12
    assert b3[16:] == [Fraction(3, 80)] * 4
    for p in (1, 2, 3):
        assert sum(refelem.basis_integrals_exact(p)) == VOL


@pytest.mark.parametrize("p", [1, 2, 3])
def test_stiffness_invariants(p):
    S = refelem.S(p)
    K = S[0, 0] + S[1, 1] + S[2, 2]
    assert np.allclose(K, K.T, atol=0)
    assert np.max(np.abs(K.sum(axis=1))) < 1e-14
    for a, b in product(range(3), repeat=2):
        assert np.allclose(S[a, b], S[b, a].T, atol=1e-15)
        assert np.max(np.abs(S[a, b].sum(axis=1))) < 1e-14
    ev = np.linalg.eigvalsh(K)
    assert abs(ev[0]) < 1e-13 and ev[1] > 1e-3       # PSD, one-dimensional kernel (constants)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_weighted_tensors_sum_to_stiffness(p):
    # sum_v l_v = 1  =>  sum_v T^{v,ab} = S^{ab}
    T = refelem.weighted_stiffness_tensors_exact(p)
    S = refelem.stiffness_tensors_exact(p)
    n = refelem.nloc(p)
    for a, b, i, j in product(range(3), range(3), range(n), range(n)):
        assert sum(T[v][a][b][i][j] for v in range(4)) == S[a][b][i][j]


@pytest.mark.parametrize("p", [1, 2, 3])
def test_partition_of_unity_and_nodality(p):
    nodes = refelem.reference_nodes(p)
    for idx, (x, y, z) in enumerate(nodes):
        vals = refelem.eval_basis_exact(p, x, y, z)
        assert vals == [Fraction(int(i == idx)) for i in range(len(nodes))]
    rng = np.random.default_rng(0)
    pts = rng.dirichlet(np.ones(4), 20)[:, 1:]
    assert np.allclose(refelem.eval_basis(p, pts).sum(axis=1), 1.0, atol=1e-14)


def test_p2_p3_kernel_and_extremes():
    # fixed spectra of the reference stiffness matrices (trace and Frobenius norm, exact)
    K2 = [[sum(refelem.stiffness_tensors_exact(2)[a][a][i][j] for a in range(3)) for j in range(10)]
          for i in range(10)]
    assert sum(K2[i][i] for i in range(10)) == Fraction(23, 5)
    assert sum(v * v for row in K2 for v in row) == Fraction(719, 150)
    K3 = [[sum(refelem.stiffness_tensors_exact(3)[a][a][i][j] for a in range(3)) for j in range(20)]
          for i in range(20)]
    assert sum(K3[i][i] for i in range(20)) == Fraction(3907, 280)
    assert sum(v * v for row in K3 for v in row) == Fraction(1566193, 62720)


@pytest.mark.parametrize("deg", [1, 2, 3, 4, 5, 6, 7, 8])
def test_conical_rule_exact(deg):
    pts, w = quadrature.conical_product_rule(deg)
    assert abs(w.sum() - 1 / 6) < 1e-15
    for a, b, c in product(range(deg + 1), repeat=3):
        if a + b + c > deg:
            continue
        got = np.sum(w * pts[:, 0] ** a * pts[:, 1] ** b * pts[:, 2] ** c)
        exact = factorial(a) * factorial(b) * factorial(c) / factorial(a + b + c + 3)
        assert abs(got - exact) <= 1e-15 + 1e-13 * exact
