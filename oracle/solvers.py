"""FP64 solvers: CG, Jacobi-CG, Chebyshev smoothing, V-cycle, MG-preconditioned CG.

Follows Section 4 of the paper (geometric multigrid: smooth, restrict the
residual, solve the coarsest problem directly, prolong the correction, smooth
again; Listing 2: 2 Chebyshev iterations per level, direct coarse solve).

Readings of the paper taken here:
* The multigrid cycle is a V(2,2) cycle used as the preconditioner of CG
  (the configuration this library targets); Listing 2's full-multigrid cycle
  with a preonly outer solver is MGHierarchy.fmg (one F-cycle: restricted
  right-hand sides, exact coarse solve, prolongation and one V-cycle per level).
* The smoother is Chebyshev on D^-1 A (Jacobi-preconditioned) over the
  interval [0.1 lmax, 1.1 lmax], degree 2, in the three-term recurrence of
  Saad, Iterative Methods for Sparse Linear Systems, Alg. 12.1.  The same
  smoother runs before and after the coarse correction, so the cycle is
  symmetric.
* Restriction is the transpose of prolongation; level operators are
  rediscretised on each mesh (for constant k this equals the Galerkin product).
* CG stops when the true residual ||b - A x|| / ||b|| <= rtol, x0 = 0.

Parity: CG against a dense solve on tiny problems, Chebyshev damping against
the closed form on sine modes, V-cycle symmetry; tests/test_oracle_solvers.py
in tests/test_oracle_solvers.py.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import assemble, patch, transfer
from .mesh import Level


def cg(A, b, rtol=1e-10, max_it=10000, M=None, x0=None, flexible=False):
    """Preconditioned CG; M(r) applies the preconditioner (None: identity).

    Returns (x, iterations, history of ||r||/||b||).  flexible=True uses the
    Polak-Ribiere beta.
    """
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - A @ x
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return x, 0, [0.0]
    z = r.copy() if M is None else M(r)
    p = z.copy()
    rz = r @ z
    hist = [np.linalg.norm(r) / nb]
    it = 0
    while hist[-1] > rtol and it < max_it:
        Ap = A @ p
        alpha = rz / (p @ Ap)
        x += alpha * p
        r_old = r
        r = r - alpha * Ap
        it += 1
        hist.append(np.linalg.norm(r) / nb)
        if hist[-1] <= rtol:
            break
        z_new = r.copy() if M is None else M(r)
        rz_new = r @ z_new
        beta = ((rz_new - (r_old @ z_new)) / rz) if flexible else rz_new / rz
        p = z_new + beta * p
        rz = rz_new
    return x, it, hist


def chebyshev_smooth(A, dinv, b, x, lmax, degree=2, lo=0.1, hi=1.1):
    """`degree` Chebyshev steps for A x = b, preconditioner diag^-1 (dinv an array) or a
    callable r -> B r (the star patches of Listing 2), on [lo*lmax, hi*lmax] (Saad Alg. 12.1).
    Returns the new x."""
    prec = dinv if callable(dinv) else (lambda v: dinv * v)
    alpha, beta = lo * lmax, hi * lmax
    theta = 0.5 * (beta + alpha)
    delta = 0.5 * (beta - alpha)
    sigma = theta / delta
    rho = 1.0 / sigma
    r = b - A @ x
    d = prec(r) / theta
    x = x.copy()
    for k in range(degree):
        x = x + d
        if k == degree - 1:
            break
        r = r - A @ d
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * prec(r)
        rho = rho_new
    return x


def lanczos_lmax(A, dinv, steps=10, seed=5):
    """Largest Ritz value of `steps` Lanczos steps on D^-1 A (D-inner product)."""
    n = A.shape[0]
    v = np.random.default_rng(seed).standard_normal(n)
    d = 1.0 / dinv
    v /= np.sqrt(v @ (d * v))
    alphas, betas = [], []
    v_prev = np.zeros(n)
    beta = 0.0
    for _ in range(steps):
        w = dinv * (A @ v)
        a = w @ (d * v)
        w = w - a * v - beta * v_prev
        alphas.append(a)
        beta = np.sqrt(max(w @ (d * w), 0.0))
        if beta == 0.0:
            break
        betas.append(beta)
        v_prev, v = v, w / beta
    k = len(alphas)
    Tm = np.diag(alphas) + np.diag(betas[:k - 1], 1) + np.diag(betas[:k - 1], -1)
    return float(np.max(np.linalg.eigvalsh(Tm)))


def pcg_lanczos_lmax(A, prec, steps=10, seed=5):
    """Largest Ritz value of B A (B = prec, symmetric positive definite) from `steps` steps of
    preconditioned CG on A e = v, v random: the CG coefficients alpha_j, beta_j define the
    Lanczos tridiagonal with diagonal 1/alpha_j + beta_{j-1}/alpha_{j-1} and off-diagonal
    sqrt(beta_j)/alpha_j (Saad, Iterative Methods for Sparse Linear Systems, 6.7.3)."""
    r = np.random.default_rng(seed).standard_normal(A.shape[0])
    z = prec(r)
    p = z.copy()
    rz = r @ z
    alphas, betas = [], []
    for it in range(steps):
        q = A @ p
        pq = p @ q
        if not pq > 0:
            break
        alphas.append(rz / pq)
        if it == steps - 1:
            break
        r = r - alphas[-1] * q
        z = prec(r)
        rz_new = r @ z
        if not rz_new > 0:
            break
        betas.append(rz_new / rz)
        rz = rz_new
        p = z + betas[-1] * p
    k = len(alphas)
    diag = [1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0) for j in range(k)]
    off = [np.sqrt(betas[j]) / alphas[j] for j in range(k - 1)]
    Tm = np.diag(diag) + np.diag(off, 1) + np.diag(off, -1)
    return float(np.max(np.linalg.eigvalsh(Tm)))


@dataclass
class MGLevel:
    level: Level
    A: sp.csr_matrix           # with boundary conditions
    dinv: np.ndarray
    lmax: float = 0.0
    P: sp.csr_matrix | None = None   # prolongation from the next coarser level


class MGHierarchy:
    """Rediscretised operators, prolongations and smoother data per level."""

    def __init__(self, levels, k_fine_vertex=None, lmax=None, eig_steps=10,
                 cheb_degree=2, cheb_lo=0.1, cheb_hi=1.1, smoother="jacobi"):
        """smoother: "jacobi" (diag^-1) or "patch" (Listing 2's additive vertex-star patches,
        oracle/patch.py) as the Chebyshev preconditioner; lambda_max of B A by Lanczos on
        D^-1 A, or by CG-Lanczos for the patches."""
        self.cheb = (cheb_degree, cheb_lo, cheb_hi)
        ks = _inject_k(levels, k_fine_vertex)
        self.levels = []
        for ell, lev in enumerate(levels):
            A = assemble.apply_bc(assemble.stiffness(lev, ks[ell]), lev.boundary)
            dinv = 1.0 / A.diagonal()
            if smoother == "patch" and ell > 0:
                pts = patch.star_patches(lev)
                inv = patch.patch_inverses(A, pts)
                dinv = (lambda v, pts=pts, inv=inv, bnd=lev.boundary: patch.apply_patch_pc(pts, inv, bnd, v))
            m = MGLevel(lev, A, dinv)
            if ell > 0:
                m.P = transfer.prolongation(levels[ell - 1], lev)
                if lmax is not None and lmax[ell] > 0:
                    m.lmax = lmax[ell]
                elif callable(dinv):
                    m.lmax = pcg_lanczos_lmax(A, dinv, eig_steps)
                else:
                    m.lmax = lanczos_lmax(A, dinv, eig_steps)
            self.levels.append(m)
        A0 = self.levels[0].A
        if A0.shape[0] <= 4000:
            lu = spla.splu(A0.tocsc())
            self.coarse_solve = lu.solve
        else:
            self.coarse_solve = lambda r: direct_solve(A0, r)

    def vcycle(self, r, ell=None):
        """One V(2,2) cycle applied to residual r on level ell: returns B r."""
        if ell is None:
            ell = len(self.levels) - 1
        if ell == 0:
            return self.coarse_solve(r)
        L = self.levels[ell]
        deg, lo, hi = self.cheb
        x = chebyshev_smooth(L.A, L.dinv, r, np.zeros_like(r), L.lmax, deg, lo, hi)
        res = r - L.A @ x
        rc = L.P.T @ res
        rc[self.levels[ell - 1].level.boundary] = 0.0
        ec = self.vcycle(rc, ell - 1)
        x = x + L.P @ ec
        x = chebyshev_smooth(L.A, L.dinv, r, x, L.lmax, deg, lo, hi)
        return x

    def solve(self, b, rtol=1e-8, max_it=200, flexible=False):
        A = self.levels[-1].A
        return cg(A, b, rtol=rtol, max_it=max_it, M=self.vcycle, flexible=flexible)

    def fmg(self, b):
        """One full-multigrid cycle as the solver (Listing 2: full multigrid with a preonly
        outer solver): the right-hand side is restricted to every level (R = P^T, boundary rows
        zero), the coarsest problem is solved exactly, and on each finer level the prolonged
        coarse solution is corrected by one V-cycle on that level's residual."""
        bs = [None] * len(self.levels)
        bs[-1] = np.asarray(b, dtype=np.float64)
        for ell in range(len(self.levels) - 1, 0, -1):
            bc = self.levels[ell].P.T @ bs[ell]
            bc[self.levels[ell - 1].level.boundary] = 0.0
            bs[ell - 1] = bc
        x = self.coarse_solve(bs[0])
        for ell in range(1, len(self.levels)):
            L = self.levels[ell]
            x = L.P @ x
            x = x + self.vcycle(bs[ell] - L.A @ x, ell)
        return x


def _inject_k(levels, k_fine_vertex):
    """Coefficient on every level by injection of the fine vertex values."""
    if k_fine_vertex is None:
        return [None] * len(levels)
    ks = [None] * len(levels)
    ks[-1] = np.asarray(k_fine_vertex, dtype=np.float64)
    for ell in range(len(levels) - 2, -1, -1):
        nf, nc = levels[ell + 1].n, levels[ell].n
        r = np.arange(nc + 1)
        kk, jj, ii = np.meshgrid(r, r, r, indexing="ij")
        fine_ids = (2 * ii) + (nf + 1) * ((2 * jj) + (nf + 1) * (2 * kk))
        ks[ell] = ks[ell + 1][fine_ids.ravel()]
    return ks


def direct_solve(A_bc: sp.csr_matrix, b: np.ndarray, rtol: float = 1e-14) -> np.ndarray:
    """Reference solution of A_bc x = b.

    Sparse LU for small systems; above 4000 unknowns, Jacobi-preconditioned CG
    to a relative residual of `rtol` (SuperLU's fill on 3-D meshes makes LU far
    slower there, and the solution is the same to rounding).
    """
    if A_bc.shape[0] <= 4000:
        return spla.splu(A_bc.tocsc()).solve(b)
    dinv = 1.0 / A_bc.diagonal()
    x, _, hist = cg(A_bc, b, rtol=rtol, max_it=20000, M=lambda r: dinv * r)
    if hist[-1] > 10 * rtol:
        raise RuntimeError(f"reference CG stalled at {hist[-1]:.3e}")
    return x
