// C ABI: argument validation on the host, then the device operations.
#include <hip/hip_runtime.h>

#include <cstring>
#include <exception>
#include <string>

#include "ops.hpp"

namespace fem {
static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
}  // namespace fem

using namespace fem;

#define FEM_REQUIRE(cond, code, msg)   \
    do {                               \
        if (!(cond)) {                 \
            fem::set_error(msg);       \
            return (code);             \
        }                              \
    } while (0)

extern "C" {

const char* fem_status_string(fem_status s) {
    switch (s) {
        case FEM_OK: return "FEM_OK";
        case FEM_WARN_NOT_CONVERGED: return "FEM_WARN_NOT_CONVERGED";
        case FEM_ERR_INVALID_ARG: return "FEM_ERR_INVALID_ARG";
        case FEM_ERR_UNSUPPORTED: return "FEM_ERR_UNSUPPORTED";
        case FEM_ERR_WORKSPACE: return "FEM_ERR_WORKSPACE";
        case FEM_ERR_HIP: return "FEM_ERR_HIP";
        case FEM_ERR_BREAKDOWN: return "FEM_ERR_BREAKDOWN";
        case FEM_ERR_STATE: return "FEM_ERR_STATE";
        default: return "FEM_UNKNOWN_STATUS";
    }
}

const char* fem_last_error(void) { return fem::g_last_error.c_str(); }

fem_status fem_mesh_create(const fem_mesh_desc* desc, fem_mesh** out) {
    FEM_REQUIRE(desc && out, FEM_ERR_INVALID_ARG, "fem_mesh_create: NULL argument");
    *out = nullptr;
    FEM_REQUIRE(desc->n >= 1, FEM_ERR_INVALID_ARG, "fem_mesh_create: n must be >= 1");
    FEM_REQUIRE(desc->degree >= 1 && desc->degree <= 3, FEM_ERR_INVALID_ARG, "fem_mesh_create: degree must be 1, 2 or 3");
    FEM_REQUIRE(desc->n_refine >= 0 && desc->n_refine <= 7, FEM_ERR_INVALID_ARG, "fem_mesh_create: n_refine must be in 0..7");
    FEM_REQUIRE(!(desc->flags & FEM_MESH_JITTER) || desc->jitter, FEM_ERR_INVALID_ARG,
                "fem_mesh_create: FEM_MESH_JITTER needs a jitter array");
    const int64_t nf = (int64_t)desc->n << desc->n_refine;
    const int64_t Lf = (int64_t)desc->degree * nf + 1;
    FEM_REQUIRE(Lf * Lf * Lf < (int64_t)0x7fffffff && 6 * nf * nf * nf * 20 < ((int64_t)1 << 40), FEM_ERR_INVALID_ARG,
                "fem_mesh_create: mesh too large for int32 dof indexing");
    fem_mesh* m = new fem_mesh();
    try {
        const fem_status st = build_mesh(*desc, *m);
        if (st != FEM_OK) {
            delete m;
            return st;
        }
    } catch (const std::exception& e) {
        delete m;
        set_error(std::string("fem_mesh_create: ") + e.what());
        return FEM_ERR_INVALID_ARG;
    }
    *out = m;
    return FEM_OK;
}

fem_status fem_mesh_device_bytes(const fem_mesh* m, size_t* bytes) {
    FEM_REQUIRE(m && bytes, FEM_ERR_INVALID_ARG, "fem_mesh_device_bytes: NULL argument");
    *bytes = m->bytes;
    return FEM_OK;
}

fem_status fem_mesh_levels(const fem_mesh* m, int32_t* n) {
    FEM_REQUIRE(m && n, FEM_ERR_INVALID_ARG, "fem_mesh_levels: NULL argument");
    *n = m->nlev;
    return FEM_OK;
}

fem_status fem_mesh_upload(fem_mesh* m, void* dev, size_t bytes, void* stream) {
    FEM_REQUIRE(m && dev, FEM_ERR_INVALID_ARG, "fem_mesh_upload: NULL argument");
    FEM_REQUIRE(((uintptr_t)dev & 255) == 0, FEM_ERR_INVALID_ARG, "fem_mesh_upload: buffer not 256-byte aligned");
    FEM_REQUIRE(bytes >= m->bytes, FEM_ERR_WORKSPACE, "fem_mesh_upload: buffer smaller than fem_mesh_device_bytes");
    hipStream_t s = (hipStream_t)stream;
    char* base = (char*)dev;
    auto put = [&](size_t off, const void* src, size_t nbytes) -> hipError_t {
        if (!nbytes) return hipSuccess;
        return hipMemcpyAsync(base + off, src, nbytes, hipMemcpyHostToDevice, s);
    };
    hipError_t e = hipSuccess;
    for (const auto& T : m->tab) {
        if (e == hipSuccess) e = put(T.d64, T.t64.data(), T.t64.size() * 8);
        if (e == hipSuccess) e = put(T.d32, T.t32.data(), T.t32.size() * 4);
    }
    if (e == hipSuccess) e = put(m->d_mref64, m->mref64.data(), m->mref64.size() * 8);
    if (e == hipSuccess) e = put(m->d_mref32, m->mref32.data(), m->mref32.size() * 4);
    if (e == hipSuccess) e = put(m->d_geo, m->geo.data(), m->geo.size() * 8);
    if (e == hipSuccess) e = put(m->d_pt_off, m->pt_off.data(), m->pt_off.size() * 4);
    if (e == hipSuccess) e = put(m->d_pt_w64, m->pt_w64.data(), m->pt_w64.size() * 8);
    if (e == hipSuccess) e = put(m->d_pt_w32, m->pt_w32.data(), m->pt_w32.size() * 4);
    if (e == hipSuccess) e = put(m->d_rs_start, m->rs_start.data(), m->rs_start.size() * 4);
    if (e == hipSuccess) e = put(m->d_rs_off, m->rs_off.data(), m->rs_off.size() * 4);
    if (e == hipSuccess) e = put(m->d_rs_w64, m->rs_w64.data(), m->rs_w64.size() * 8);
    if (e == hipSuccess) e = put(m->d_rs_w32, m->rs_w32.data(), m->rs_w32.size() * 4);
    for (const auto& L : m->lev) {
        if (e == hipSuccess) e = put(L.d_map, L.map.data(), L.map.size() * 4);
        if (e == hipSuccess) e = put(L.d_G64, L.G64.data(), L.G64.size() * 8);
        if (e == hipSuccess) e = put(L.d_G32, L.G32.data(), L.G32.size() * 4);
        if (e == hipSuccess) e = put(L.d_vsoa, L.vsoa.data(), L.vsoa.size() * 8);
        if (e == hipSuccess) e = put(L.d_rs_lin, L.rs_lin.data(), L.rs_lin.size() * 4);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        set_error(std::string("fem_mesh_upload: ") + hipGetErrorString(e));
        return FEM_ERR_HIP;
    }
    int dev_id = -1;
    if (hipGetDevice(&dev_id) != hipSuccess) dev_id = -1;
    m->dev = base;
    m->device = dev_id;
    return FEM_OK;
}

fem_status fem_mesh_info(const fem_mesh* m, int32_t level, fem_level_info* info) {
    FEM_REQUIRE(m && info, FEM_ERR_INVALID_ARG, "fem_mesh_info: NULL argument");
    FEM_REQUIRE(level >= 0 && level < m->nlev, FEM_ERR_INVALID_ARG, "fem_mesh_info: level out of range");
    const HostLevel& L = m->lev[level];
    info->n_cells = L.C;
    info->n_dofs = L.N;
    info->n_interior = L.NI;
    info->n_vertices = L.NV;
    info->n = L.n;
    info->degree = L.p;
    info->brick = L.B;
    info->geometry = action_geometry(*m, level);
    return FEM_OK;
}

fem_status fem_mesh_dof_lattice(const fem_mesh* m, int32_t level, int32_t* ijk) {
    FEM_REQUIRE(m && ijk, FEM_ERR_INVALID_ARG, "fem_mesh_dof_lattice: NULL argument");
    FEM_REQUIRE(level >= 0 && level < m->nlev, FEM_ERR_INVALID_ARG, "fem_mesh_dof_lattice: level out of range");
    const int64_t L = m->lev[level].L;
    int64_t g = 0;
    for (int64_t k = 0; k < L; ++k)
        for (int64_t j = 0; j < L; ++j)
            for (int64_t i = 0; i < L; ++i, ++g) {
                ijk[3 * g] = (int32_t)i;
                ijk[3 * g + 1] = (int32_t)j;
                ijk[3 * g + 2] = (int32_t)k;
            }
    return FEM_OK;
}

fem_status fem_mesh_vertex_coords(const fem_mesh* m, int32_t level, double* xyz) {
    FEM_REQUIRE(m && xyz, FEM_ERR_INVALID_ARG, "fem_mesh_vertex_coords: NULL argument");
    FEM_REQUIRE(level >= 0 && level < m->nlev, FEM_ERR_INVALID_ARG, "fem_mesh_vertex_coords: level out of range");
    std::memcpy(xyz, m->lev[level].vxyz.data(), m->lev[level].vxyz.size() * sizeof(double));
    return FEM_OK;
}

void fem_mesh_destroy(fem_mesh* m) { delete m; }

static fem_status check_common(const fem_mesh* m, int32_t level, int dtype, const char* fn) {
    FEM_REQUIRE(m, FEM_ERR_INVALID_ARG, std::string(fn) + ": NULL mesh");
    FEM_REQUIRE(level >= 0 && level < m->nlev, FEM_ERR_INVALID_ARG, std::string(fn) + ": level out of range");
    FEM_REQUIRE(dtype == FEM_F64 || dtype == FEM_F32, FEM_ERR_INVALID_ARG, std::string(fn) + ": bad dtype");
    FEM_REQUIRE(m->dev != nullptr, FEM_ERR_STATE, std::string(fn) + ": mesh not uploaded");
    return FEM_OK;
}

static int row_mode_of(uint32_t flags) {
    return flags == FEM_BC_NONE ? ROW_NONE : flags == FEM_BC_ZERO_ROWS ? ROW_ZERO : ROW_IDENTITY;
}

fem_status fem_apply_laplacian_axpby(const fem_mesh* m, int32_t level, fem_dtype dtype, const void* k,
                                     const void* x, double alpha, const void* z, double beta, void* y,
                                     uint32_t flags, void* stream) {
    fem_status st = check_common(m, level, dtype, "fem_apply_laplacian");
    if (st) return st;
    FEM_REQUIRE(x && y, FEM_ERR_INVALID_ARG, "fem_apply_laplacian: NULL vector");
    FEM_REQUIRE(x != y, FEM_ERR_INVALID_ARG, "fem_apply_laplacian: x and y must differ");
    FEM_REQUIRE(beta == 0.0 || z, FEM_ERR_INVALID_ARG, "fem_apply_laplacian: z is NULL with beta != 0");
    FEM_REQUIRE(z != x || beta == 0.0, FEM_ERR_INVALID_ARG, "fem_apply_laplacian: z must not alias x");
    FEM_REQUIRE(flags <= FEM_BC_ZERO_ROWS, FEM_ERR_INVALID_ARG, "fem_apply_laplacian: bad flags");
    const int rm = row_mode_of(flags);
    const bool mask = flags != FEM_BC_NONE && flags != FEM_BC_ZERO_ROWS;
    hipStream_t s = (hipStream_t)stream;
    if (dtype == FEM_F64) {
        ScatterIO<double> io;
        io.x = (const double*)x;
        io.k = (const double*)k;
        io.y = (double*)y;
        io.z = (const double*)z;
        io.alpha = alpha;
        io.beta = beta;
        io.row_mode = rm;
        io.xid = (const double*)x;
        io.mask_cols = mask;
        return run_scatter<double>(*m, level, K_APPLY, k != nullptr, io, s);
    }
    ScatterIO<float> io;
    io.x = (const float*)x;
    io.k = (const float*)k;
    io.y = (float*)y;
    io.z = (const float*)z;
    io.alpha = alpha;
    io.beta = beta;
    io.row_mode = rm;
    io.xid = (const float*)x;
    io.mask_cols = mask;
    return run_scatter<float>(*m, level, K_APPLY, k != nullptr, io, s);
}

fem_status fem_apply_laplacian(const fem_mesh* m, int32_t level, fem_dtype dtype, const void* k, const void* x,
                               void* y, uint32_t flags, void* stream) {
    return fem_apply_laplacian_axpby(m, level, dtype, k, x, 1.0, nullptr, 0.0, y, flags, stream);
}

fem_status fem_apply_laplacian_noalloc(const fem_mesh* m, int32_t level, fem_dtype dtype, const void* k,
                                      const void* x, void* y, uint32_t flags, void* stream) {
    fem_status st = check_common(m, level, dtype, "fem_apply_laplacian_noalloc");
    if (st) return st;
    FEM_REQUIRE(x && y, FEM_ERR_INVALID_ARG, "fem_apply_laplacian_noalloc: NULL vector");
    FEM_REQUIRE(x != y, FEM_ERR_INVALID_ARG, "fem_apply_laplacian_noalloc: x and y must differ");
    FEM_REQUIRE(flags <= FEM_BC_ZERO_ROWS, FEM_ERR_INVALID_ARG, "fem_apply_laplacian_noalloc: bad flags");
    int dev = -1;
    FEM_REQUIRE(hipGetDevice(&dev) == hipSuccess && dev == m->device, FEM_ERR_INVALID_ARG,
                "fem_apply_laplacian_noalloc: the current device is not the mesh's device");
    void* scr = nullptr;
    size_t scr_bytes = 0;
    st = noalloc_scratch(&scr, &scr_bytes);
    if (st) return st;
    const int rm = row_mode_of(flags);
    const bool mask = flags != FEM_BC_NONE && flags != FEM_BC_ZERO_ROWS;
    hipStream_t s = (hipStream_t)stream;
    if (dtype == FEM_F64) {
        ScatterIO<double> io;
        io.x = (const double*)x;
        io.k = (const double*)k;
        io.y = (double*)y;
        io.row_mode = rm;
        io.xid = (const double*)x;
        io.mask_cols = mask;
        io.slots = scr;
        io.slots_bytes = scr_bytes;
        return run_scatter<double>(*m, level, K_APPLY, k != nullptr, io, s);
    }
    ScatterIO<float> io;
    io.x = (const float*)x;
    io.k = (const float*)k;
    io.y = (float*)y;
    io.row_mode = rm;
    io.xid = (const float*)x;
    io.mask_cols = mask;
    io.slots = scr;
    io.slots_bytes = scr_bytes;
    return run_scatter<float>(*m, level, K_APPLY, k != nullptr, io, s);
}

fem_status fem_apply_mass(const fem_mesh* m, int32_t level, fem_dtype dtype, const void* x, void* y, uint32_t flags,
                          void* stream) {
    fem_status st = check_common(m, level, dtype, "fem_apply_mass");
    if (st) return st;
    FEM_REQUIRE(x && y && x != y, FEM_ERR_INVALID_ARG, "fem_apply_mass: NULL or aliased vectors");
    FEM_REQUIRE(flags <= FEM_BC_ZERO_ROWS, FEM_ERR_INVALID_ARG, "fem_apply_mass: bad flags");
    const int rm = row_mode_of(flags);
    const bool mask = flags == FEM_BC_IDENTITY;
    hipStream_t s = (hipStream_t)stream;
    if (dtype == FEM_F64) {
        ScatterIO<double> io;
        io.x = (const double*)x;
        io.y = (double*)y;
        io.row_mode = rm;
        io.xid = (const double*)x;
        io.mask_cols = mask;
        return run_scatter<double>(*m, level, K_MASS, false, io, s);
    }
    ScatterIO<float> io;
    io.x = (const float*)x;
    io.y = (float*)y;
    io.row_mode = rm;
    io.xid = (const float*)x;
    io.mask_cols = mask;
    return run_scatter<float>(*m, level, K_MASS, false, io, s);
}

fem_status fem_assemble_diagonal(const fem_mesh* m, int32_t level, fem_dtype dtype, const void* k, void* d,
                                 void* stream) {
    fem_status st = check_common(m, level, dtype, "fem_assemble_diagonal");
    if (st) return st;
    FEM_REQUIRE(d, FEM_ERR_INVALID_ARG, "fem_assemble_diagonal: NULL output");
    hipStream_t s = (hipStream_t)stream;
    if (dtype == FEM_F64) {
        ScatterIO<double> io;
        io.k = (const double*)k;
        io.y = (double*)d;
        io.row_mode = ROW_ONE;
        return run_scatter<double>(*m, level, K_DIAG, k != nullptr, io, s);
    }
    ScatterIO<float> io;
    io.k = (const float*)k;
    io.y = (float*)d;
    io.row_mode = ROW_ONE;
    return run_scatter<float>(*m, level, K_DIAG, k != nullptr, io, s);
}

fem_status fem_prolong(const fem_mesh* m, int32_t fine_level, fem_dtype dtype, const void* xc, void* xf,
                       void* stream) {
    fem_status st = check_common(m, fine_level, dtype, "fem_prolong");
    if (st) return st;
    FEM_REQUIRE(fine_level >= 1, FEM_ERR_INVALID_ARG, "fem_prolong: fine_level must be >= 1");
    FEM_REQUIRE(xc && xf && xc != xf, FEM_ERR_INVALID_ARG, "fem_prolong: NULL or aliased vectors");
    hipStream_t s = (hipStream_t)stream;
    if (dtype == FEM_F64) return run_prolong<double>(*m, fine_level, (const double*)xc, (double*)xf, s);
    return run_prolong<float>(*m, fine_level, (const float*)xc, (float*)xf, s);
}

fem_status fem_restrict(const fem_mesh* m, int32_t fine_level, fem_dtype dtype, const void* rf, void* rc,
                        void* stream) {
    fem_status st = check_common(m, fine_level, dtype, "fem_restrict");
    if (st) return st;
    FEM_REQUIRE(fine_level >= 1, FEM_ERR_INVALID_ARG, "fem_restrict: fine_level must be >= 1");
    FEM_REQUIRE(rf && rc && rf != rc, FEM_ERR_INVALID_ARG, "fem_restrict: NULL or aliased vectors");
    hipStream_t s = (hipStream_t)stream;
    if (dtype == FEM_F64) return run_restrict<double>(*m, fine_level, (const double*)rf, (double*)rc, s);
    return run_restrict<float>(*m, fine_level, (const float*)rf, (float*)rc, s);
}

fem_status fem_adjoint_grad_k(const fem_mesh* m, int32_t level, const double* k, const double* u,
                              const double* lam, double* grad, void* stream) {
    (void)k;
    fem_status st = check_common(m, level, FEM_F64, "fem_adjoint_grad_k");
    if (st) return st;
    FEM_REQUIRE(u && lam && grad, FEM_ERR_INVALID_ARG, "fem_adjoint_grad_k: NULL vector");
    FEM_REQUIRE((const void*)grad != (const void*)u && (const void*)grad != (const void*)lam, FEM_ERR_INVALID_ARG,
                "fem_adjoint_grad_k: grad aliases an input");
    ScatterIO<double> io;
    io.x = u;
    io.x2 = lam;
    io.y = grad;
    io.row_mode = ROW_NONE;
    return run_scatter<double>(*m, level, K_GRAD, false, io, (hipStream_t)stream);
}

fem_status fem_patch_bytes(const fem_mesh* m, int32_t level, fem_dtype dtype, size_t* bytes) {
    FEM_REQUIRE(m && bytes, FEM_ERR_INVALID_ARG, "fem_patch_bytes: NULL argument");
    FEM_REQUIRE(level >= 0 && level < m->nlev, FEM_ERR_INVALID_ARG, "fem_patch_bytes: level out of range");
    FEM_REQUIRE(dtype == FEM_F64 || dtype == FEM_F32, FEM_ERR_INVALID_ARG, "fem_patch_bytes: bad dtype");
    std::string why;
    FEM_REQUIRE(patch_supported(m->lev[level], why), FEM_ERR_UNSUPPORTED, "fem_patch_bytes: " + why);
    *bytes = patch_bytes(m->lev[level], dtype == FEM_F64 ? 8 : 4);
    return FEM_OK;
}

fem_status fem_patch_setup(const fem_mesh* m, int32_t level, fem_dtype dtype, const double* k, void* patch,
                           size_t bytes, void* stream) {
    fem_status st = check_common(m, level, dtype, "fem_patch_setup");
    if (st) return st;
    std::string why;
    FEM_REQUIRE(patch_supported(m->lev[level], why), FEM_ERR_UNSUPPORTED, "fem_patch_setup: " + why);
    const size_t need = patch_bytes(m->lev[level], dtype == FEM_F64 ? 8 : 4);
    FEM_REQUIRE(patch && bytes >= need, FEM_ERR_WORKSPACE, "fem_patch_setup: patch buffer NULL or too small");
    return dtype == FEM_F64 ? patch_setup<double>(*m, level, k, patch, (hipStream_t)stream)
                            : patch_setup<float>(*m, level, k, patch, (hipStream_t)stream);
}

fem_status fem_apply_patch(const fem_mesh* m, int32_t level, fem_dtype dtype, void* patch, size_t bytes,
                           const void* r, void* z, void* stream) {
    fem_status st = check_common(m, level, dtype, "fem_apply_patch");
    if (st) return st;
    std::string why;
    FEM_REQUIRE(patch_supported(m->lev[level], why), FEM_ERR_UNSUPPORTED, "fem_apply_patch: " + why);
    const size_t need = patch_bytes(m->lev[level], dtype == FEM_F64 ? 8 : 4);
    FEM_REQUIRE(patch && bytes >= need, FEM_ERR_WORKSPACE, "fem_apply_patch: patch buffer NULL or too small");
    FEM_REQUIRE(r && z, FEM_ERR_INVALID_ARG, "fem_apply_patch: NULL vector");
    FEM_REQUIRE(r != z, FEM_ERR_INVALID_ARG, "fem_apply_patch: r and z must differ");
    if (dtype == FEM_F64)
        return patch_apply<double>(*m, level, patch, (const double*)r, (double*)z, (hipStream_t)stream);
    return patch_apply<float>(*m, level, patch, (const float*)r, (float*)z, (hipStream_t)stream);
}

}  // extern "C"
