"""Writes p3_48_vark_solution.txt: sampled values of the oracle's solution of the variable-
coefficient P3 problem at full size, for the GPU solve parity test.

Problem (the paper's Poisson problem of Section 2, eq. 4 with a coefficient, Listing 1's
degree-3 space and Dirichlet conditions; the solver of Section 4, Listing 2): -div(k grad u) = 1
on the unit cube, 6^3 x 6 tetrahedra refined three times to 48^3 x 6 (3,048,625 P3 dofs),
k = exp(g) the P1 field of 16 seeded Fourier modes (fem_inputs.k_exp_fourier, seed 1),
b = P_I M 1 (boundary rows zero).  Solved by the oracle's FP64 CG preconditioned with its own
4-level V-cycle (oracle.solvers.MGHierarchy) to relative residual 1e-13.

Only oracle/ and the seeded input generators are used.  Run: python tests/golden/make_p3_48_vark_solution.py
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import fem_inputs  # noqa: E402
from oracle import assemble, solvers  # noqa: E402
from oracle import mesh as om  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "p3_48_vark_solution.txt")
N0, REFINE, P = 6, 3, 3
RTOL = 1e-13


def sample_indices(n_dofs: int, L: int) -> np.ndarray:
    """Seeded random dofs plus dofs next to the boundary, at the corners and on brick planes."""
    rng = np.random.default_rng(12)
    idx = rng.integers(0, n_dofs, 1200).tolist()
    pts = [(1, 1, 1), (L - 2, L - 2, L - 2), (1, L // 2, L - 2), (L // 2, L // 2, L // 2), (12, 12, 12),
           (24, 36, 12), (13, 12, 11), (72, 71, 1), (0, 5, 7), (L - 1, 64, 3)]
    idx += [i + L * (j + L * k) for i, j, k in pts]
    face = rng.integers(1, L - 1, (200, 3))
    face[:, 0] = rng.choice([1, 2, 12, 24, 36, L - 3, L - 2], 200)
    idx += [int(i + L * (j + L * k)) for i, j, k in face]
    return np.unique(np.array(idx, dtype=np.int64))


def main():
    t0 = time.time()
    levels = om.hierarchy(N0, REFINE, P)
    lev = levels[-1]
    k = fem_inputs.k_exp_fourier(lev.vert_xyz)
    b = assemble.mass(lev) @ np.ones(lev.n_dofs)
    b[lev.boundary] = 0.0
    print(f"mesh and rhs {time.time() - t0:.1f} s", flush=True)
    mg = solvers.MGHierarchy(levels, k)
    print(f"hierarchy {time.time() - t0:.1f} s, lambda_max {[round(L.lmax, 6) for L in mg.levels[1:]]}", flush=True)
    u, its, hist = mg.solve(b, rtol=RTOL, max_it=400)
    A = mg.levels[-1].A
    res = np.linalg.norm(b - A @ u) / np.linalg.norm(b)
    print(f"solve {time.time() - t0:.1f} s, {its} iterations, true relative residual {res:.3e}", flush=True)
    assert res <= 1e-12
    L = P * lev.n + 1
    idx = sample_indices(lev.n_dofs, L)
    with open(OUT, "w") as fh:
        fh.write("# Oracle FP64 solution of -div(k grad u) = 1, P3 on 48^3 x 6 tetrahedra (6^3 refined 3x),\n")
        fh.write("# k = exp(g) (fem_inputs.k_exp_fourier, seed 1), b = P_I M 1; oracle MG-CG to rel residual 1e-13\n")
        fh.write("# (paper Section 2 eq. 4 with Listing 1's P3 space and Dirichlet conditions; Section 4 solver).\n")
        fh.write("# Written by tests/golden/make_p3_48_vark_solution.py (oracle only).  Dof index: lexicographic\n")
        fh.write("# lattice order I + L (J + L K), L = 145.\n")
        fh.write(f"n_dofs {lev.n_dofs}\n")
        fh.write(f"norm_u {np.linalg.norm(u):.17e}\n")
        fh.write(f"norm_b {np.linalg.norm(b):.17e}\n")
        fh.write(f"true_rel_residual {res:.3e}\n")
        fh.write(f"iterations {its}\n")
        for i in idx:
            fh.write(f"{int(i)} {u[i]:.17e}\n")
    print(f"wrote {OUT} ({len(idx)} sampled dofs), {time.time() - t0:.1f} s")


if __name__ == "__main__":
    main()
