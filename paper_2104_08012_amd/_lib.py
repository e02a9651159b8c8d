"""ctypes binding of libfem.so (argument marshalling only).

The library must have been built in-tree (``python -m paper_2104_08012_amd.build`` or
``__graft_entry__.build()``); importing anything that needs it raises if it is missing.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfem.so")

FEM_OK = 0
FEM_WARN_NOT_CONVERGED = 1
FEM_ERR_INVALID_ARG = -1
FEM_ERR_UNSUPPORTED = -2
FEM_ERR_WORKSPACE = -3
FEM_ERR_HIP = -4
FEM_ERR_BREAKDOWN = -5
FEM_ERR_STATE = -6

FEM_F64 = 0
FEM_F32 = 1
FEM_BC_IDENTITY = 0
FEM_BC_NONE = 1
FEM_BC_ZERO_ROWS = 2
FEM_MESH_JITTER = 1
FEM_PREC_FP64 = 0
FEM_PREC_MIXED = 1
FEM_COARSE_AUTO = 0
FEM_COARSE_DENSE = 1
FEM_COARSE_NESTED = 2
FEM_COARSE_DENSE_F32 = 3
FEM_PC_MG = 0
FEM_PC_JACOBI = 1
FEM_SMOOTHER_JACOBI = 0
FEM_SMOOTHER_PATCH = 1


class MeshDesc(C.Structure):
    _fields_ = [("n", C.c_int32), ("n_refine", C.c_int32), ("degree", C.c_int32),
                ("flags", C.c_uint32), ("jitter", C.POINTER(C.c_double))]


class LevelInfo(C.Structure):
    _fields_ = [("n_cells", C.c_int64), ("n_dofs", C.c_int64), ("n_interior", C.c_int64),
                ("n_vertices", C.c_int64), ("n", C.c_int32), ("degree", C.c_int32),
                ("brick", C.c_int32), ("geometry", C.c_int32)]


class SolveOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("max_it", C.c_int32), ("precision", C.c_int32),
                ("n_levels_used", C.c_int32), ("cheb_degree", C.c_int32),
                ("cheb_lo", C.c_double), ("cheb_hi", C.c_double), ("eig_iters", C.c_int32),
                ("coarse_method", C.c_int32), ("lambda_max_override", C.POINTER(C.c_double)),
                ("coarse_rtol", C.c_double), ("replace_every", C.c_int32), ("flexible", C.c_int32),
                ("history", C.POINTER(C.c_double)), ("history_cap", C.c_int32),
                ("preconditioner", C.c_int32), ("level_timing", C.c_int32),
                ("smoother", C.c_int32)]


class SolveStats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("coarse_iterations", C.c_int32),
                ("rel_residual_true", C.c_double), ("setup_ms", C.c_double),
                ("solve_ms", C.c_double), ("coarse_ms", C.c_double),
                ("level_ms", C.c_double * 8), ("lambda_max", C.c_double * 8)]


_vp = C.c_void_p
_i32 = C.c_int32
_st = C.c_int32

SIGNATURES = {
    "fem_status_string": (C.c_char_p, [_st]),
    "fem_last_error": (C.c_char_p, []),
    "fem_mesh_create": (_st, [C.POINTER(MeshDesc), C.POINTER(_vp)]),
    "fem_mesh_device_bytes": (_st, [_vp, C.POINTER(C.c_size_t)]),
    "fem_mesh_upload": (_st, [_vp, _vp, C.c_size_t, _vp]),
    "fem_mesh_levels": (_st, [_vp, C.POINTER(_i32)]),
    "fem_mesh_info": (_st, [_vp, _i32, C.POINTER(LevelInfo)]),
    "fem_mesh_dof_lattice": (_st, [_vp, _i32, _vp]),
    "fem_mesh_vertex_coords": (_st, [_vp, _i32, _vp]),
    "fem_mesh_destroy": (None, [_vp]),
    "fem_apply_laplacian": (_st, [_vp, _i32, _i32, _vp, _vp, _vp, C.c_uint32, _vp]),
    "fem_apply_laplacian_axpby": (_st, [_vp, _i32, _i32, _vp, _vp, C.c_double, _vp, C.c_double, _vp,
                                        C.c_uint32, _vp]),
    "fem_apply_laplacian_noalloc": (_st, [_vp, _i32, _i32, _vp, _vp, _vp, C.c_uint32, _vp]),
    "fem_apply_mass": (_st, [_vp, _i32, _i32, _vp, _vp, C.c_uint32, _vp]),
    "fem_assemble_diagonal": (_st, [_vp, _i32, _i32, _vp, _vp, _vp]),
    "fem_prolong": (_st, [_vp, _i32, _i32, _vp, _vp, _vp]),
    "fem_restrict": (_st, [_vp, _i32, _i32, _vp, _vp, _vp]),
    "fem_solve_opts_default": (None, [C.POINTER(SolveOpts)]),
    "fem_solve_workspace_bytes": (_st, [_vp, C.POINTER(SolveOpts), C.POINTER(C.c_size_t)]),
    "fem_solver_create": (_st, [_vp, C.POINTER(SolveOpts), _vp, C.c_size_t, C.POINTER(_vp)]),
    "fem_solver_setup": (_st, [_vp, _vp, _vp]),
    "fem_solver_solve": (_st, [_vp, _vp, _vp, C.POINTER(SolveStats), _vp]),
    "fem_solver_vcycle": (_st, [_vp, _vp, _vp, _vp]),
    "fem_solver_fmg": (_st, [_vp, _vp, _vp, C.POINTER(SolveStats), _vp]),
    "fem_solver_set_level_timing": (_st, [_vp, _i32]),
    "fem_solver_destroy": (None, [_vp]),
    "fem_mg_cg_solve": (_st, [_vp, _vp, _vp, _vp, C.POINTER(SolveOpts), _vp, C.c_size_t,
                              C.POINTER(SolveStats), _vp]),
    "fem_adjoint_grad_k": (_st, [_vp, _i32, _vp, _vp, _vp, _vp, _vp]),
    "fem_csr_create": (_st, [_vp, _i32, C.POINTER(_vp)]),
    "fem_csr_info": (_st, [_vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_size_t)]),
    "fem_csr_pattern": (_st, [_vp, _vp, _vp]),
    "fem_csr_upload": (_st, [_vp, _vp, C.c_size_t, _vp]),
    "fem_csr_assemble": (_st, [_vp, _i32, _vp, _vp, _vp]),
    "fem_csr_spmv": (_st, [_vp, _i32, _vp, _vp, _vp, _vp]),
    "fem_csr_destroy": (None, [_vp]),
    "fem_patch_bytes": (_st, [_vp, _i32, _i32, C.POINTER(C.c_size_t)]),
    "fem_patch_setup": (_st, [_vp, _i32, _i32, _vp, _vp, C.c_size_t, _vp]),
    "fem_apply_patch": (_st, [_vp, _i32, _i32, _vp, C.c_size_t, _vp, _vp, _vp]),
}

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(there is no fallback implementation)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class FemError(RuntimeError):
    def __init__(self, status: int, where: str):
        L = lib()
        msg = L.fem_last_error().decode()
        name = L.fem_status_string(status).decode()
        super().__init__(f"{where}: {name} ({status}): {msg}")
        self.status = status


def check(status: int, where: str, allow_warning: bool = False) -> int:
    if status < 0 or (status > 0 and not allow_warning):
        raise FemError(status, where)
    return status
