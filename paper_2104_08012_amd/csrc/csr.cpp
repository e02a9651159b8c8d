// Assembled operator: host construction of the CSR pattern of A_bc on one mesh level and of
// each stored entry's list of element-matrix contributions; C entry points.
//
// The pattern is the union, per row (dof), of the dofs of the cells containing it.  Entry (r, c)
// of A receives a_K[i][j] from every cell K with dof(K, i) = r and dof(K, j) = c; the host lists
// these (as positions (i nloc + j) C + K in the entry-major element-matrix buffer) in ascending
// cell order, so the device sum has a fixed order.  Dirichlet rows become identity rows and
// Dirichlet columns zero (symmetric elimination, paper §2 with the DirichletBC of Listing 1).
#include <algorithm>
#include <cstring>
#include <string>

#include "csr.hpp"

using namespace fem;

namespace {

fem_status build_csr(const fem_mesh& m, int level, fem_csr& A) {
    const HostLevel& L = m.lev[level];
    const int nl = L.nloc;
    const int64_t C = L.C, N = L.N;
    if (C * nl * nl >= (int64_t)1 << 31 || N >= (int64_t)1 << 31) {
        set_error("fem_csr_create: level too large for 32-bit contribution indices");
        return FEM_ERR_UNSUPPORTED;
    }
    auto dof = [&](int64_t c, int i) { return (int64_t)((uint32_t)L.map[(size_t)i * C + c] & 0x7fffffffu); };
    auto bnd = [&](int64_t c, int i) { return L.map[(size_t)i * C + c] < 0; };
    // dof -> (cell, local node) incidence, ascending cell order
    std::vector<int64_t> ip(N + 1, 0);
    for (int64_t c = 0; c < C; ++c)
        for (int i = 0; i < nl; ++i) ++ip[dof(c, i) + 1];
    for (int64_t r = 0; r < N; ++r) ip[r + 1] += ip[r];
    std::vector<int64_t> fill(ip.begin(), ip.end() - 1);
    std::vector<int64_t> inc((size_t)C * nl);
    for (int64_t c = 0; c < C; ++c)
        for (int i = 0; i < nl; ++i) inc[fill[dof(c, i)]++] = c * nl + i;
    std::vector<uint8_t> isb(N, 0);
    for (int64_t c = 0; c < C; ++c)
        for (int i = 0; i < nl; ++i)
            if (bnd(c, i)) isb[dof(c, i)] = 1;
    // pattern
    A.n = N;
    A.row_ptr.assign(N + 1, 0);
    std::vector<int32_t> cols;
    std::vector<int32_t> buf;
    for (int64_t r = 0; r < N; ++r) {
        buf.clear();
        for (int64_t t = ip[r]; t < ip[r + 1]; ++t) {
            const int64_t c = inc[t] / nl;
            for (int j = 0; j < nl; ++j) buf.push_back((int32_t)dof(c, j));
        }
        std::sort(buf.begin(), buf.end());
        buf.erase(std::unique(buf.begin(), buf.end()), buf.end());
        cols.insert(cols.end(), buf.begin(), buf.end());
        if ((int64_t)cols.size() >= (int64_t)1 << 31) {
            set_error("fem_csr_create: more than 2^31 stored entries");
            return FEM_ERR_UNSUPPORTED;
        }
        A.row_ptr[r + 1] = (int32_t)cols.size();
    }
    A.col.swap(cols);
    A.nnz = (int64_t)A.col.size();
    // contributions: count, then fill in the same (row, ascending cell, j) order
    auto pos = [&](int64_t r, int64_t c) {
        const int32_t* b = A.col.data() + A.row_ptr[r];
        const int32_t* e = A.col.data() + A.row_ptr[r + 1];
        return (int64_t)(std::lower_bound(b, e, (int32_t)c) - A.col.data());
    };
    A.cptr.assign(A.nnz + 1, 0);
    for (int64_t r = 0; r < N; ++r)
        for (int64_t t = ip[r]; t < ip[r + 1]; ++t) {
            const int64_t c = inc[t] / nl;
            for (int j = 0; j < nl; ++j) ++A.cptr[pos(r, dof(c, j)) + 1];
        }
    for (int64_t e = 0; e < A.nnz; ++e) A.cptr[e + 1] += A.cptr[e];
    A.ncontrib = A.cptr[A.nnz];
    A.cidx.assign(A.ncontrib, 0);
    std::vector<int64_t> f2(A.cptr.begin(), A.cptr.end() - 1);
    for (int64_t r = 0; r < N; ++r)
        for (int64_t t = ip[r]; t < ip[r + 1]; ++t) {
            const int64_t c = inc[t] / nl;
            const int i = (int)(inc[t] % nl);
            for (int j = 0; j < nl; ++j) A.cidx[f2[pos(r, dof(c, j))]++] = (int32_t)((int64_t)(i * nl + j) * C + c);
        }
    A.flag.assign(A.nnz, CSR_SUM);
    for (int64_t r = 0; r < N; ++r)
        for (int32_t e = A.row_ptr[r]; e < A.row_ptr[r + 1]; ++e) {
            const int64_t c = A.col[e];
            if (isb[r]) A.flag[e] = (c == r) ? CSR_ONE : CSR_ZERO;
            else if (isb[c]) A.flag[e] = CSR_ZERO;
        }
    // device layout
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t o = off;
        off = align256(off + b);
        return o;
    };
    A.d_rp = take((N + 1) * 4);
    A.d_col = take(A.nnz * 4);
    A.d_cptr = take((A.nnz + 1) * 8);
    A.d_cidx = take(A.ncontrib * 4);
    A.d_flag = take(A.nnz);
    A.d_elem = take((size_t)C * nl * nl * 8);
    A.bytes = off;
    return FEM_OK;
}

}  // namespace

#define CSR_REQUIRE(cond, code, msg) \
    do {                             \
        if (!(cond)) {               \
            set_error(msg);          \
            return (code);           \
        }                            \
    } while (0)

extern "C" {

fem_status fem_csr_create(const fem_mesh* m, int32_t level, fem_csr** out) {
    CSR_REQUIRE(m && out, FEM_ERR_INVALID_ARG, "fem_csr_create: NULL argument");
    CSR_REQUIRE(level >= 0 && level < m->nlev, FEM_ERR_INVALID_ARG, "fem_csr_create: level out of range");
    *out = nullptr;
    fem_csr* A = new fem_csr();
    A->m = m;
    A->level = level;
    fem_status st = FEM_OK;
    try {
        st = build_csr(*m, level, *A);
    } catch (const std::exception& e) {
        set_error(std::string("fem_csr_create: ") + e.what());
        st = FEM_ERR_INVALID_ARG;
    }
    if (st) {
        delete A;
        return st;
    }
    *out = A;
    return FEM_OK;
}

fem_status fem_csr_info(const fem_csr* A, int64_t* n_rows, int64_t* nnz, size_t* device_bytes) {
    CSR_REQUIRE(A && n_rows && nnz && device_bytes, FEM_ERR_INVALID_ARG, "fem_csr_info: NULL argument");
    *n_rows = A->n;
    *nnz = A->nnz;
    *device_bytes = A->bytes;
    return FEM_OK;
}

fem_status fem_csr_pattern(const fem_csr* A, int32_t* row_ptr, int32_t* col) {
    CSR_REQUIRE(A && row_ptr && col, FEM_ERR_INVALID_ARG, "fem_csr_pattern: NULL argument");
    std::memcpy(row_ptr, A->row_ptr.data(), (A->n + 1) * 4);
    std::memcpy(col, A->col.data(), A->nnz * 4);
    return FEM_OK;
}

fem_status fem_csr_upload(fem_csr* A, void* dev, size_t bytes, void* stream) {
    CSR_REQUIRE(A && dev, FEM_ERR_INVALID_ARG, "fem_csr_upload: NULL argument");
    CSR_REQUIRE(((uintptr_t)dev & 255) == 0, FEM_ERR_INVALID_ARG, "fem_csr_upload: buffer not 256-byte aligned");
    CSR_REQUIRE(bytes >= A->bytes, FEM_ERR_WORKSPACE, "fem_csr_upload: buffer smaller than the device bytes");
    hipStream_t s = (hipStream_t)stream;
    char* base = (char*)dev;
    hipError_t e = hipMemcpyAsync(base + A->d_rp, A->row_ptr.data(), (A->n + 1) * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(base + A->d_col, A->col.data(), A->nnz * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(base + A->d_cptr, A->cptr.data(), (A->nnz + 1) * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(base + A->d_cidx, A->cidx.data(), A->ncontrib * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(base + A->d_flag, A->flag.data(), A->nnz, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        set_error(std::string("fem_csr_upload: ") + hipGetErrorString(e));
        return FEM_ERR_HIP;
    }
    A->dev = base;
    return FEM_OK;
}

fem_status fem_csr_assemble(fem_csr* A, fem_dtype dtype, const double* k, void* values, void* stream) {
    CSR_REQUIRE(A && values, FEM_ERR_INVALID_ARG, "fem_csr_assemble: NULL argument");
    CSR_REQUIRE(A->dev, FEM_ERR_STATE, "fem_csr_assemble: not uploaded");
    CSR_REQUIRE(A->m->dev, FEM_ERR_STATE, "fem_csr_assemble: mesh not uploaded");
    CSR_REQUIRE(dtype == FEM_F64 || dtype == FEM_F32, FEM_ERR_INVALID_ARG, "fem_csr_assemble: bad dtype");
    const fem_mesh& m = *A->m;
    const HostLevel& L = m.lev[A->level];
    hipStream_t s = (hipStream_t)stream;
    const Tabulation& T = m.tab[k ? 1 : 0];
    double* E = reinterpret_cast<double*>(A->dev + A->d_elem);
    csr_elem_launch(L.nloc, L.C, L.n, L.p, L.L, dptr<int32_t>(m, L.d_map), dptr<double>(m, L.d_G64),
                    dptr<double>(m, T.d64), T.nq, k, E, s);
    const int64_t* cptr = reinterpret_cast<const int64_t*>(A->dev + A->d_cptr);
    const int32_t* cidx = reinterpret_cast<const int32_t*>(A->dev + A->d_cidx);
    const uint8_t* flag = reinterpret_cast<const uint8_t*>(A->dev + A->d_flag);
    if (dtype == FEM_F64) csr_gather_launch<double>(A->nnz, cptr, cidx, flag, E, (double*)values, s);
    else csr_gather_launch<float>(A->nnz, cptr, cidx, flag, E, (float*)values, s);
    return check_launch("fem_csr_assemble");
}

fem_status fem_csr_spmv(const fem_csr* A, fem_dtype dtype, const void* values, const void* x, void* y, void* stream) {
    CSR_REQUIRE(A && values && x && y && x != y, FEM_ERR_INVALID_ARG, "fem_csr_spmv: NULL or aliased argument");
    CSR_REQUIRE(A->dev, FEM_ERR_STATE, "fem_csr_spmv: not uploaded");
    CSR_REQUIRE(dtype == FEM_F64 || dtype == FEM_F32, FEM_ERR_INVALID_ARG, "fem_csr_spmv: bad dtype");
    hipStream_t s = (hipStream_t)stream;
    const int32_t* rp = reinterpret_cast<const int32_t*>(A->dev + A->d_rp);
    const int32_t* col = reinterpret_cast<const int32_t*>(A->dev + A->d_col);
    const int lanes = A->m->p == 1 ? 4 : 8;   // P1 rows ~15 entries, P2 ~29, P3 ~50 (measured best)
    if (dtype == FEM_F64)
        csr_spmv_launch<double>(A->n, lanes, rp, col, (const double*)values, (const double*)x, (double*)y, s);
    else
        csr_spmv_launch<float>(A->n, lanes, rp, col, (const float*)values, (const float*)x, (float*)y, s);
    return check_launch("fem_csr_spmv");
}

void fem_csr_destroy(fem_csr* A) { delete A; }

}  // extern "C"
