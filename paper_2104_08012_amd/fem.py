"""Python surface of the library: meshes, operator applications, solves, gradients.

Thin marshalling over the C ABI (include/fem.h).  PyTorch provides device memory and
streams; every computation runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib as L
from ._lib import check, lib

_DT = {torch.float64: L.FEM_F64, torch.float32: L.FEM_F32}
_BC = {"identity": L.FEM_BC_IDENTITY, "none": L.FEM_BC_NONE, "zero_rows": L.FEM_BC_ZERO_ROWS}


def _stream(device=None) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else t.data_ptr()


def _need(t: torch.Tensor, n: int, dtype: torch.dtype, what: str):
    if not t.is_cuda or t.dtype != dtype or t.numel() != n or not t.is_contiguous():
        raise ValueError(f"{what}: expected contiguous {dtype} CUDA tensor with {n} entries, "
                         f"got {t.dtype} {tuple(t.shape)} on {t.device}")


class Mesh:
    """Tetrahedral unit-cube hierarchy (n^3 cubes x 6, refined n_refine times), P_degree."""

    def __init__(self, n: int, n_refine: int, degree: int, jitter: np.ndarray | None = None,
                 device: str | torch.device = "cuda", upload: bool = True):
        desc = L.MeshDesc()
        desc.n, desc.n_refine, desc.degree = n, n_refine, degree
        self._jit = None
        if jitter is not None:
            self._jit = np.ascontiguousarray(jitter, dtype=np.float64)
            if self._jit.shape != ((n + 1) ** 3, 3):
                raise ValueError("jitter must have shape ((n+1)^3, 3)")
            desc.flags = L.FEM_MESH_JITTER
            desc.jitter = self._jit.ctypes.data_as(C.POINTER(C.c_double))
        h = C.c_void_p()
        check(lib().fem_mesh_create(C.byref(desc), C.byref(h)), "fem_mesh_create")
        self._h = h
        self.n0, self.n_refine, self.degree = n, n_refine, degree
        nl = C.c_int32()
        check(lib().fem_mesh_levels(h, C.byref(nl)), "fem_mesh_levels")
        self.n_levels = nl.value
        self.levels = [self.info(i) for i in range(self.n_levels)]
        self.buffer = None
        if upload:
            self.upload(device)

    @property
    def handle(self):
        return self._h

    def device_bytes(self) -> int:
        b = C.c_size_t()
        check(lib().fem_mesh_device_bytes(self._h, C.byref(b)), "fem_mesh_device_bytes")
        return b.value

    def upload(self, device="cuda"):
        nbytes = self.device_bytes()
        self.device = torch.device(device)
        self.buffer = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        check(lib().fem_mesh_upload(self._h, _ptr(self.buffer), nbytes, _stream(self.device)),
              "fem_mesh_upload")

    def info(self, level: int) -> dict:
        i = L.LevelInfo()
        check(lib().fem_mesh_info(self._h, level, C.byref(i)), "fem_mesh_info")
        return {"n_cells": i.n_cells, "n_dofs": i.n_dofs, "n_interior": i.n_interior,
                "n_vertices": i.n_vertices, "n": i.n, "degree": i.degree, "brick": i.brick,
                "geometry": ("cell", "vertex", "table")[i.geometry]}

    def _lev(self, level: int) -> int:
        return level % self.n_levels

    def dof_lattice(self, level: int = -1) -> np.ndarray:
        level = self._lev(level)
        out = np.empty((self.levels[level]["n_dofs"], 3), dtype=np.int32)
        check(lib().fem_mesh_dof_lattice(self._h, level, out.ctypes.data), "fem_mesh_dof_lattice")
        return out

    def vertex_coords(self, level: int = -1) -> np.ndarray:
        level = self._lev(level)
        out = np.empty((self.levels[level]["n_vertices"], 3), dtype=np.float64)
        check(lib().fem_mesh_vertex_coords(self._h, level, out.ctypes.data), "fem_mesh_vertex_coords")
        return out

    def n_dofs(self, level: int = -1) -> int:
        return self.levels[self._lev(level)]["n_dofs"]

    def n_vertices(self, level: int = -1) -> int:
        return self.levels[self._lev(level)]["n_vertices"]

    # ---- operator applications (stream-ordered, asynchronous) ----
    def apply(self, x: torch.Tensor, k: torch.Tensor | None = None, level: int = -1, bc: str = "identity",
              out: torch.Tensor | None = None, alpha: float = 1.0, z: torch.Tensor | None = None,
              beta: float = 0.0) -> torch.Tensor:
        level = self._lev(level)
        n = self.n_dofs(level)
        _need(x, n, x.dtype, "apply x")
        if k is not None:
            _need(k, self.n_vertices(level), x.dtype, "apply k")
        y = torch.empty_like(x) if out is None else out
        _need(y, n, x.dtype, "apply out")
        if z is not None:
            _need(z, n, x.dtype, "apply z")
        check(lib().fem_apply_laplacian_axpby(self._h, level, _DT[x.dtype], _ptr(k), _ptr(x), alpha, _ptr(z),
                                              beta, _ptr(y), _BC[bc], _stream(x.device)),
              "fem_apply_laplacian")
        return y

    def mass(self, x: torch.Tensor, level: int = -1, bc: str = "none", out=None) -> torch.Tensor:
        level = self._lev(level)
        _need(x, self.n_dofs(level), x.dtype, "mass x")
        y = torch.empty_like(x) if out is None else out
        check(lib().fem_apply_mass(self._h, level, _DT[x.dtype], _ptr(x), _ptr(y), _BC[bc], _stream(x.device)),
              "fem_apply_mass")
        return y

    def diagonal(self, k: torch.Tensor | None = None, level: int = -1, dtype=torch.float64) -> torch.Tensor:
        level = self._lev(level)
        d = torch.empty(self.n_dofs(level), dtype=dtype, device=self.device)
        if k is not None:
            _need(k, self.n_vertices(level), dtype, "diagonal k")
        check(lib().fem_assemble_diagonal(self._h, level, _DT[dtype], _ptr(k), _ptr(d), _stream(d.device)),
              "fem_assemble_diagonal")
        return d

    def prolong(self, xc: torch.Tensor, xf: torch.Tensor, fine_level: int) -> torch.Tensor:
        _need(xc, self.n_dofs(fine_level - 1), xc.dtype, "prolong coarse")
        _need(xf, self.n_dofs(fine_level), xc.dtype, "prolong fine")
        check(lib().fem_prolong(self._h, fine_level, _DT[xc.dtype], _ptr(xc), _ptr(xf), _stream(xc.device)),
              "fem_prolong")
        return xf

    def restrict(self, rf: torch.Tensor, fine_level: int, out=None) -> torch.Tensor:
        _need(rf, self.n_dofs(fine_level), rf.dtype, "restrict fine")
        rc = torch.empty(self.n_dofs(fine_level - 1), dtype=rf.dtype, device=rf.device) if out is None else out
        check(lib().fem_restrict(self._h, fine_level, _DT[rf.dtype], _ptr(rf), _ptr(rc), _stream(rf.device)),
              "fem_restrict")
        return rc

    def adjoint_grad_k(self, u: torch.Tensor, lam: torch.Tensor, level: int = -1, out=None) -> torch.Tensor:
        level = self._lev(level)
        _need(u, self.n_dofs(level), torch.float64, "grad u")
        _need(lam, self.n_dofs(level), torch.float64, "grad lambda")
        g = torch.empty(self.n_vertices(level), dtype=torch.float64, device=u.device) if out is None else out
        check(lib().fem_adjoint_grad_k(self._h, level, None, _ptr(u), _ptr(lam), _ptr(g), _stream(u.device)),
              "fem_adjoint_grad_k")
        return g

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                lib().fem_mesh_destroy(self._h)
                self._h = None
        except Exception:
            pass


class PatchPreconditioner:
    """Additive vertex-star patch preconditioner of one P2 mesh level (Section 2, Listing 2: star
    patches around vertices): z = sum_v R_v^T A_v^{-1} R_v r on interior dofs, z_B = r_B.  The
    star inverses and partial results live in a device buffer owned by this object."""

    def __init__(self, mesh: Mesh, level: int = -1, k: torch.Tensor | None = None, dtype=torch.float64):
        self.mesh = mesh
        self.level = mesh._lev(level)
        self.dtype = dtype
        nb = C.c_size_t()
        check(lib().fem_patch_bytes(mesh.handle, self.level, _DT[dtype], C.byref(nb)), "fem_patch_bytes")
        self.nbytes = nb.value
        self.buffer = torch.empty(max(256, self.nbytes), dtype=torch.uint8, device=mesh.device)
        self.setup(k)

    def setup(self, k: torch.Tensor | None = None):
        if k is not None:
            _need(k, self.mesh.n_vertices(self.level), torch.float64, "patch k")
        check(lib().fem_patch_setup(self.mesh.handle, self.level, _DT[self.dtype], _ptr(k), _ptr(self.buffer),
                                    self.nbytes, _stream(self.mesh.device)), "fem_patch_setup")

    def apply(self, r: torch.Tensor, out=None) -> torch.Tensor:
        n = self.mesh.n_dofs(self.level)
        _need(r, n, self.dtype, "patch r")
        z = torch.empty_like(r) if out is None else out
        _need(z, n, self.dtype, "patch z")
        check(lib().fem_apply_patch(self.mesh.handle, self.level, _DT[self.dtype], _ptr(self.buffer), self.nbytes,
                                    _ptr(r), _ptr(z), _stream(r.device)), "fem_apply_patch")
        return z


class CsrOperator:
    """Assembled CSR matrix of A_bc(k) on one mesh level (host pattern, device values)."""

    def __init__(self, mesh: Mesh, level: int = -1, upload: bool = True):
        self.mesh = mesh
        self.level = mesh._lev(level)
        h = C.c_void_p()
        check(lib().fem_csr_create(mesh.handle, self.level, C.byref(h)), "fem_csr_create")
        self._h = h
        n, nnz, nb = C.c_int64(), C.c_int64(), C.c_size_t()
        check(lib().fem_csr_info(h, C.byref(n), C.byref(nnz), C.byref(nb)), "fem_csr_info")
        self.n_rows, self.nnz, self.device_bytes = n.value, nnz.value, nb.value
        self.buffer = None
        if upload:
            self.buffer = torch.empty(max(256, self.device_bytes), dtype=torch.uint8, device=mesh.device)
            check(lib().fem_csr_upload(h, _ptr(self.buffer), self.device_bytes, _stream(mesh.device)),
                  "fem_csr_upload")

    def pattern(self):
        rp = np.empty(self.n_rows + 1, dtype=np.int32)
        col = np.empty(self.nnz, dtype=np.int32)
        check(lib().fem_csr_pattern(self._h, rp.ctypes.data, col.ctypes.data), "fem_csr_pattern")
        return rp, col

    def assemble(self, k: torch.Tensor | None = None, dtype=torch.float64, out=None) -> torch.Tensor:
        if k is not None:
            _need(k, self.mesh.n_vertices(self.level), torch.float64, "csr k")
        vals = torch.empty(self.nnz, dtype=dtype, device=self.mesh.device) if out is None else out
        _need(vals, self.nnz, dtype, "csr values")
        check(lib().fem_csr_assemble(self._h, _DT[dtype], _ptr(k), _ptr(vals), _stream(vals.device)),
              "fem_csr_assemble")
        return vals

    def spmv(self, values: torch.Tensor, x: torch.Tensor, out=None) -> torch.Tensor:
        _need(values, self.nnz, values.dtype, "csr values")
        _need(x, self.n_rows, values.dtype, "spmv x")
        y = torch.empty_like(x) if out is None else out
        _need(y, self.n_rows, values.dtype, "spmv y")
        check(lib().fem_csr_spmv(self._h, _DT[values.dtype], _ptr(values), _ptr(x), _ptr(y), _stream(x.device)),
              "fem_csr_spmv")
        return y

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                lib().fem_csr_destroy(self._h)
                self._h = None
        except Exception:
            pass


@dataclass
class SolveOptions:
    rtol: float = 1e-8
    max_it: int = 200
    precision: str = "fp64"        # "fp64" or "mixed"
    n_levels_used: int = 0
    cheb_degree: int = 2
    cheb_lo: float = 0.1
    cheb_hi: float = 1.1
    eig_iters: int = 10
    coarse_method: str = "auto"    # "auto", "dense", "nested", "dense_f32" (mixed only: FP32-stored inverse)
    lambda_max: list | None = None
    coarse_rtol: float = 1e-10
    replace_every: int = 25
    flexible: bool | None = None   # default: Polak-Ribiere beta in mixed precision
    history_cap: int = 1000
    preconditioner: str = "mg"     # "mg" or "jacobi"
    level_timing: bool = False     # per-level V-cycle times in SolveResult.level_ms (adds events)
    smoother: str = "jacobi"       # "jacobi" or "patch" (vertex-star patches, P2)

    def to_c(self):
        o = L.SolveOpts()
        lib().fem_solve_opts_default(C.byref(o))
        o.rtol, o.max_it = self.rtol, self.max_it
        o.precision = L.FEM_PREC_MIXED if self.precision == "mixed" else L.FEM_PREC_FP64
        o.n_levels_used = self.n_levels_used
        o.cheb_degree, o.cheb_lo, o.cheb_hi = self.cheb_degree, self.cheb_lo, self.cheb_hi
        o.eig_iters = self.eig_iters
        o.coarse_method = {"auto": L.FEM_COARSE_AUTO, "dense": L.FEM_COARSE_DENSE,
                           "nested": L.FEM_COARSE_NESTED, "dense_f32": L.FEM_COARSE_DENSE_F32}[self.coarse_method]
        keep = []
        if self.lambda_max is not None:
            arr = (C.c_double * len(self.lambda_max))(*self.lambda_max)
            o.lambda_max_override = C.cast(arr, C.POINTER(C.c_double))
            keep.append(arr)
        o.coarse_rtol = self.coarse_rtol
        o.replace_every = self.replace_every
        flex = (self.precision == "mixed") if self.flexible is None else self.flexible
        o.flexible = 1 if flex else 0
        hist = (C.c_double * max(1, self.history_cap))()
        o.history = C.cast(hist, C.POINTER(C.c_double))
        o.history_cap = self.history_cap
        o.preconditioner = L.FEM_PC_JACOBI if self.preconditioner == "jacobi" else L.FEM_PC_MG
        o.smoother = {"jacobi": L.FEM_SMOOTHER_JACOBI, "patch": L.FEM_SMOOTHER_PATCH}[self.smoother]
        o.level_timing = 1 if self.level_timing else 0
        keep.append(hist)
        return o, keep, hist


@dataclass
class SolveResult:
    iterations: int
    rel_residual_true: float
    setup_ms: float
    solve_ms: float
    coarse_ms: float
    level_ms: list
    lambda_max: list
    history: list
    coarse_iterations: int
    status: int
    extra: dict = field(default_factory=dict)


class Solver:
    """MG-preconditioned CG bound to a mesh, options and a device workspace."""

    def __init__(self, mesh: Mesh, opts: SolveOptions | None = None):
        self.mesh = mesh
        self.opts = opts or SolveOptions()
        self._copts, self._keep, self._hist = self.opts.to_c()
        nb = C.c_size_t()
        check(lib().fem_solve_workspace_bytes(mesh.handle, C.byref(self._copts), C.byref(nb)),
              "fem_solve_workspace_bytes")
        self.workspace = torch.empty(max(256, nb.value), dtype=torch.uint8, device=mesh.device)
        h = C.c_void_p()
        check(lib().fem_solver_create(mesh.handle, C.byref(self._copts), _ptr(self.workspace), nb.value,
                                      C.byref(h)), "fem_solver_create")
        self._h = h
        self.k = None

    def setup(self, k: torch.Tensor | None = None):
        if k is not None:
            _need(k, self.mesh.n_vertices(-1), torch.float64, "solver k")
        self.k = k
        check(lib().fem_solver_setup(self._h, _ptr(k), _stream(self.mesh.device)), "fem_solver_setup")
        return self

    def solve(self, b: torch.Tensor, x: torch.Tensor | None = None, allow_not_converged: bool = False):
        n = self.mesh.n_dofs(-1)
        _need(b, n, torch.float64, "solve b")
        x = torch.zeros_like(b) if x is None else x
        _need(x, n, torch.float64, "solve x")
        st = L.SolveStats()
        status = lib().fem_solver_solve(self._h, _ptr(b), _ptr(x), C.byref(st), _stream(b.device))
        check(status, "fem_solver_solve", allow_warning=allow_not_converged)
        it = st.iterations
        res = SolveResult(it, st.rel_residual_true, st.setup_ms, st.solve_ms, st.coarse_ms,
                          list(st.level_ms), list(st.lambda_max),
                          [self._hist[i] for i in range(min(it + 1, self.opts.history_cap))],
                          st.coarse_iterations, status)
        return x, res

    def set_level_timing(self, on: bool):
        """Per-level V-cycle times (SolveResult.level_ms, coarse_ms) for later solves."""
        check(lib().fem_solver_set_level_timing(self._h, 1 if on else 0), "fem_solver_set_level_timing")
        return self

    def fmg(self, b: torch.Tensor, x: torch.Tensor | None = None):
        """One full-multigrid cycle as the solver (the paper's Listing 2 configuration)."""
        n = self.mesh.n_dofs(-1)
        _need(b, n, torch.float64, "fmg b")
        x = torch.empty_like(b) if x is None else x
        _need(x, n, torch.float64, "fmg x")
        st = L.SolveStats()
        check(lib().fem_solver_fmg(self._h, _ptr(b), _ptr(x), C.byref(st), _stream(b.device)), "fem_solver_fmg")
        res = SolveResult(1, st.rel_residual_true, st.setup_ms, st.solve_ms, st.coarse_ms, list(st.level_ms),
                          list(st.lambda_max), [], st.coarse_iterations, 0)
        return x, res

    def vcycle(self, r: torch.Tensor, z: torch.Tensor | None = None) -> torch.Tensor:
        z = torch.empty_like(r) if z is None else z
        check(lib().fem_solver_vcycle(self._h, _ptr(r), _ptr(z), _stream(r.device)), "fem_solver_vcycle")
        return z

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                lib().fem_solver_destroy(self._h)
                self._h = None
        except Exception:
            pass
