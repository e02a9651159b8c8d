"""Seeded synthetic inputs shared by the HIP path, the tests and the oracle.

This module holds no finite element arithmetic: it draws random numbers and
evaluates closed-form functions at points handed to it.  Everything here is an
*input* (a vector, a coefficient field, a manufactured solution, a mesh
perturbation); nothing here discretises, assembles or solves.

Seed conventions (numpy.random.default_rng):
  0  random vectors x ~ U(-1, 1) for operator actions
  1  coefficient field g for the variable-coefficient P3 workload
  2  reference coefficient k_ref for the adjoint workload
  3  observation noise
  4  finite-difference directions
  6  coarse-mesh vertex jitter
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "uniform_vector", "fourier_field_g", "k_exp_fourier", "sin3_u", "sin3_f",
    "paper_u", "paper_f", "vertex_lattice", "jitter_offsets", "noise", "fd_directions",
]


def uniform_vector(n: int, seed: int = 0, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """x ~ U(lo, hi)^n in float64."""
    return np.random.default_rng(seed).uniform(lo, hi, n)


def fourier_field_g(points: np.ndarray, seed: int = 1, modes: int = 16) -> np.ndarray:
    """g(x) = sum_m a_m cos(2 pi W_m . x + phase_m).

    W_m ~ U(1,4)^3, xi_m ~ N(0,1), phase_m ~ U(0, 2 pi), a_m = xi_m / |W_m|^2:
    16 random Fourier modes with wavevectors in [1,4]^3 and amplitudes
    N(0,1)/|w|^2, drawn in that order from one generator.
    """
    rng = np.random.default_rng(seed)
    W = rng.uniform(1.0, 4.0, (modes, 3))
    xi = rng.standard_normal(modes)
    phase = rng.uniform(0.0, 2.0 * math.pi, modes)
    a = xi / np.sum(W * W, axis=1)
    pts = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    arg = 2.0 * math.pi * (pts @ W.T) + phase[None, :]
    return np.cos(arg) @ a


def k_exp_fourier(points: np.ndarray, seed: int = 1) -> np.ndarray:
    """k = exp(g) evaluated at the given points (vertex values of a P1 field)."""
    return np.exp(fourier_field_g(points, seed))


def sin3_u(points: np.ndarray) -> np.ndarray:
    """u = sin(pi x) sin(pi y) sin(pi z)."""
    p = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    return np.sin(math.pi * p[:, 0]) * np.sin(math.pi * p[:, 1]) * np.sin(math.pi * p[:, 2])


def sin3_f(points: np.ndarray) -> np.ndarray:
    """f = 3 pi^2 sin(pi x) sin(pi y) sin(pi z), so that -lap(u) = f for sin3_u."""
    return 3.0 * math.pi ** 2 * sin3_u(points)


def paper_u(points: np.ndarray, a: float = 1.0, b: float = 2.0) -> np.ndarray:
    """Manufactured solution of the paper's Poisson example (Section 2, eq. 3)."""
    p = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    x, y, z = p[:, 0], p[:, 1], p[:, 2]
    return (np.sin(math.pi * x) * np.tan(math.pi * x / 4.0)
            * np.sin(a * math.pi * y) * np.sin(b * math.pi * z))


def paper_f(points: np.ndarray, a: float = 1.0, b: float = 2.0) -> np.ndarray:
    """Right-hand side of the paper's Poisson example (Section 2, eq. 2)."""
    p = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    x, y, z = p[:, 0], p[:, 1], p[:, 2]
    bracket = (2.0 * np.cos(math.pi * x) - np.cos(math.pi * x / 2.0)
               - 2.0 * (a * a + b * b) * np.sin(math.pi * x) * np.tan(math.pi * x / 4.0))
    return -(math.pi ** 2) / 2.0 * bracket * np.sin(a * math.pi * y) * np.sin(b * math.pi * z)


def vertex_lattice(n: int) -> np.ndarray:
    """Integer coordinates (i, j, k) of the (n+1)^3 vertices, x fastest."""
    r = np.arange(n + 1)
    k, j, i = np.meshgrid(r, r, r, indexing="ij")
    return np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)


def jitter_offsets(n: int, amp: float, seed: int = 6) -> np.ndarray:
    """Per-vertex displacements for the coarsest Kuhn(n) mesh, in units of h.

    Interior vertices move by U(-amp, amp) in each coordinate; boundary
    vertices stay put so the domain is still the unit cube.  Shape
    ((n+1)^3, 3), vertex order x fastest.  Multiply by h = 1/n for lengths.
    """
    ijk = vertex_lattice(n)
    d = np.random.default_rng(seed).uniform(-amp, amp, ijk.shape)
    boundary = np.any((ijk == 0) | (ijk == n), axis=1)
    d[boundary] = 0.0
    return d


def noise(n: int, seed: int = 3) -> np.ndarray:
    """xi ~ N(0,1)^n."""
    return np.random.default_rng(seed).standard_normal(n)


def fd_directions(nv: int, count: int = 20, seed: int = 4) -> np.ndarray:
    """count directions d ~ N(0,1)^nv, each scaled to max-norm 1."""
    d = np.random.default_rng(seed).standard_normal((count, nv))
    return d / np.max(np.abs(d), axis=1, keepdims=True)
