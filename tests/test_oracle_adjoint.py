"""Pins for the oracle's adjoint gradient: the linearity identity
<g, k> = -lam^T b, central finite differences and a Taylor remainder test."""
import numpy as np
import pytest

import fem_inputs
from oracle import adjoint, assemble
from oracle import mesh as om


def _problem(n=3, p=2, jit=True):
    lev = om.single_level(n, p, fem_inputs.jitter_offsets(n, 0.15) if jit else None)
    k_ref = fem_inputs.k_exp_fourier(lev.vert_xyz, seed=2)
    b = assemble.mass(lev) @ np.ones(lev.n_dofs)
    b[lev.boundary] = 0
    u_ref, _ = adjoint.solve_state(lev, k_ref, b)
    xi = fem_inputs.noise(lev.n_dofs)
    u_obs = u_ref + 0.01 * np.max(np.abs(u_ref)) * xi
    u_obs[lev.boundary] = 0
    return lev, b, u_obs


@pytest.mark.parametrize("p", [1, 2, 3])
def test_linearity_identity(p):
    lev, b, u_obs = _problem(p=p)
    k = fem_inputs.k_exp_fourier(lev.vert_xyz, seed=1)
    J, g, u, lam = adjoint.gradient(lev, k, b, u_obs)
    assert abs(g @ k + lam @ b) <= 1e-11 * abs(lam @ b)


@pytest.mark.parametrize("p", [1, 2])
def test_central_differences(p):
    lev, b, u_obs = _problem(p=p)
    k0 = np.ones(lev.n_vertices)
    J, g, _, _ = adjoint.gradient(lev, k0, b, u_obs)
    eps = 1e-6
    for d in fem_inputs.fd_directions(lev.n_vertices, 5):
        Jp = adjoint.objective(lev, adjoint.solve_state(lev, k0 + eps * d, b)[0], u_obs)
        Jm = adjoint.objective(lev, adjoint.solve_state(lev, k0 - eps * d, b)[0], u_obs)
        fd = (Jp - Jm) / (2 * eps)
        assert abs(fd - g @ d) <= 1e-5 * abs(g @ d)


def test_taylor_remainder_rate():
    lev, b, u_obs = _problem(p=2)
    k0 = np.ones(lev.n_vertices)
    J0, g, _, _ = adjoint.gradient(lev, k0, b, u_obs)
    d = fem_inputs.fd_directions(lev.n_vertices, 1)[0]
    res = []
    for eps in (1e-2, 5e-3, 2.5e-3):
        Je = adjoint.objective(lev, adjoint.solve_state(lev, k0 + eps * d, b)[0], u_obs)
        res.append(abs(Je - J0 - eps * (g @ d)))
    rates = np.log2(np.array(res[:-1]) / np.array(res[1:]))
    assert np.all(rates > 1.9), rates
