// Launchers for the cell-wise kernels (stiffness action, diagonal, mass, transfers, adjoint
// gradient): fill the kernel arguments from the mesh's device tables and dispatch the template
// instance for the degree, brick size, coefficient kind and precision.
#include <cmath>
#include <mutex>

#include "ops.hpp"
#include "cube.hpp"
#include "lattice.hpp"
#include "scatter.hpp"

namespace fem {

// Interface partial sums of fem_apply_laplacian_noalloc: a file-scope device array, one copy per
// GPU the library runs on, held until the process ends.  In host code its name is a host-side
// stand-in: kernels receive the device address looked up by noalloc_scratch.
constexpr size_t kNoallocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kNoallocScratchBytes];

fem_status noalloc_scratch(void** ptr, size_t* bytes) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        set_error("fem_apply_laplacian_noalloc: no current HIP device");
        return FEM_ERR_HIP;
    }
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error(std::string("fem_apply_laplacian_noalloc: scratch address lookup failed: ") +
                      hipGetErrorString(e));
            return FEM_ERR_HIP;
        }
        addr[dev] = p;
    }
    *ptr = addr[dev];
    *bytes = kNoallocScratchBytes;
    return FEM_OK;
}

namespace {

template <int P, int B, bool KV, bool GEO, typename T>
void launch_cube(const SArgs<T>& a, int64_t nbricks, hipStream_t s) {
    const int R = a.nb / a.nbx;
    const unsigned grid = (unsigned)(nbricks / R);
    if constexpr (P <= 2) {
        if (R == 4) { hipLaunchKernelGGL((k_cube_apply<P, B, 4, KV, GEO, T>), dim3(grid), dim3(4 * 64), 0, s, a); return; }
        if (R == 2) { hipLaunchKernelGGL((k_cube_apply<P, B, 2, KV, GEO, T>), dim3(grid), dim3(2 * 64), 0, s, a); return; }
    }
    hipLaunchKernelGGL((k_cube_apply<P, B, 1, KV, GEO, T>), dim3(grid), dim3(64), 0, s, a);
}

template <int KIND, typename T, int P, int B, bool KV>
void launch_main(const SArgs<T>& a, int64_t nbricks, hipStream_t s) {
    if constexpr (KIND == K_APPLY && P == 3 && B == 4) {
        // P3 on 4-cube bricks: dofs addressed by lattice point (see lattice.hpp)
        if (a.lattice) {
            if (a.geo) hipLaunchKernelGGL((k_lattice_apply<P, KV, true, T>), dim3((unsigned)nbricks), dim3(brick_threads(B)), 0, s, a);
            else hipLaunchKernelGGL((k_lattice_apply<P, KV, false, T>), dim3((unsigned)nbricks), dim3(brick_threads(B)), 0, s, a);
            return;
        }
    }
    if constexpr (KIND == K_APPLY && P <= 2 && B == 4) {
        // one thread per cube for the low degrees (see cube.hpp), where the level has the cube
        // data; R = nb / nbx bricks along x per workgroup
        if (a.vxyz) {
            if (a.geo) launch_cube<P, B, KV, true, T>(a, nbricks, s);
            else launch_cube<P, B, KV, false, T>(a, nbricks, s);
            return;
        }
    }
    {
        hipLaunchKernelGGL((k_brick<KIND, P, B, KV, T>), dim3((unsigned)nbricks), dim3(brick_threads(B)), 0, s, a);
    }
}

template <int KIND, typename T, int P, int B>
void launch_kv(bool kv, const SArgs<T>& a, int64_t nbricks, hipStream_t s) {
    if constexpr (KIND == K_APPLY || KIND == K_DIAG) {
        if (kv) { launch_main<KIND, T, P, B, true>(a, nbricks, s); return; }
    }
    launch_main<KIND, T, P, B, false>(a, nbricks, s);
}

template <int KIND, typename T, int P>
void launch_b(int B, bool kv, const SArgs<T>& a, int64_t nbricks, hipStream_t s) {
    if (B == 4) launch_kv<KIND, T, P, 4>(kv, a, nbricks, s);
    else if (B == 2) launch_kv<KIND, T, P, 2>(kv, a, nbricks, s);
    else launch_kv<KIND, T, P, 1>(kv, a, nbricks, s);
}

template <int KIND, typename T>
void launch_p(int P, int B, bool kv, const SArgs<T>& a, int64_t nbricks, hipStream_t s) {
    if (P == 1) launch_b<KIND, T, 1>(B, kv, a, nbricks, s);
    else if (P == 2) launch_b<KIND, T, 2>(B, kv, a, nbricks, s);
    else launch_b<KIND, T, 3>(B, kv, a, nbricks, s);
}

template <typename T, int PO>
void launch_fix_b(int B, const SArgs<T>& a, const FixGeom& fg, hipStream_t s) {
    const unsigned grid = (fg.total + 255) / 256;
    const int R = a.nb / a.nbx;
    if constexpr (PO <= 2) {
        if (B == 4 && R == 4) { hipLaunchKernelGGL((k_fixup<PO, 4, 4, T>), dim3(grid), dim3(256), 0, s, a, fg); return; }
        if (B == 4 && R == 2) { hipLaunchKernelGGL((k_fixup<PO, 4, 2, T>), dim3(grid), dim3(256), 0, s, a, fg); return; }
    }
    if (B == 4) hipLaunchKernelGGL((k_fixup<PO, 4, 1, T>), dim3(grid), dim3(256), 0, s, a, fg);
    else if (B == 2) hipLaunchKernelGGL((k_fixup<PO, 2, 1, T>), dim3(grid), dim3(256), 0, s, a, fg);
    else hipLaunchKernelGGL((k_fixup<PO, 1, 1, T>), dim3(grid), dim3(256), 0, s, a, fg);
}

template <typename T>
void launch_fix(int PO, int B, const SArgs<T>& a, const FixGeom& fg, hipStream_t s) {
    if (PO == 1) launch_fix_b<T, 1>(B, a, fg, s);
    else if (PO == 2) launch_fix_b<T, 2>(B, a, fg, s);
    else launch_fix_b<T, 3>(B, a, fg, s);
}

template <typename T>
const T* tab_ptr(const fem_mesh& m, int kvar);
template <>
const double* tab_ptr<double>(const fem_mesh& m, int kvar) { return dptr<double>(m, m.tab[kvar].d64); }
template <>
const float* tab_ptr<float>(const fem_mesh& m, int kvar) { return dptr<float>(m, m.tab[kvar].d32); }

template <typename T>
size_t G_off(const HostLevel& L);
template <>
size_t G_off<double>(const HostLevel& L) { return L.d_G64; }
template <>
size_t G_off<float>(const HostLevel& L) { return L.d_G32; }

template <typename T>
size_t mref_off(const fem_mesh& m) { return sizeof(T) == 8 ? m.d_mref64 : m.d_mref32; }

template <int KIND, typename T>
fem_status run_kind(const fem_mesh& m, int level, bool kvar, const ScatterIO<T>& io, hipStream_t s) {
    // level: the mesh level whose cells the kernel loops over
    const HostLevel& L = m.lev[level];
    const int po = (KIND == K_GRAD) ? 1 : m.p;
    SArgs<T> a{};
    a.n = L.n;
    a.nb = L.nb;
    a.Lout = po * L.n + 1;
    a.C = L.C;
    a.map = dptr<int32_t>(m, L.d_map);
    a.G = dptr<T>(m, G_off<T>(L));
    a.tab = tab_ptr<T>(m, (KIND == K_GRAD) ? 1 : (kvar ? 1 : 0));
    a.aux = (KIND == K_MASS) ? dptr<T>(m, mref_off<T>(m)) : nullptr;
    a.slots = io.slots ? static_cast<T*>(io.slots) : const_cast<T*>(dptr<T>(m, L.d_slots));
    a.mask_cols = io.mask_cols;
    a.x = io.x;
    a.x2 = io.x2;
    a.k = io.k;
    a.y = io.y;
    a.z = io.z;
    a.alpha = (T)io.alpha;
    a.beta = (T)io.beta;
    a.row_mode = io.row_mode;
    a.xid = io.xid;
    a.vxyz = L.cube ? dptr<double>(m, L.d_vsoa) : nullptr;
    a.nv = (uint32_t)L.NV;
    // geometry from the coarsest level's table once a brick of cubes lies inside one coarsest cube
    const bool geo = KIND == K_APPLY && action_geometry(m, level) == FEM_GEOM_TABLE;
    a.geo = geo ? dptr<double>(m, m.d_geo) : nullptr;
    a.lattice = KIND == K_APPLY && L.B == 4 && m.p == 3;
    a.geo_shift = level;
    a.geo_scale = std::ldexp(1.0, -level);
    // the P1/P2 cube kernel merges R = 4 (or 2) bricks along x in one workgroup; the interface
    // numbering then has bricks of span R p B along x (iface.hpp)
    const int R = (KIND == K_APPLY && m.p <= 2 && L.B == 4 && L.cube) ? (L.nb % 4 == 0 ? 4 : L.nb % 2 == 0 ? 2 : 1) : 1;
    a.nbx = L.nb / R;
    const int64_t Lo = a.Lout, nb = L.nb, nbx = a.nbx, np = Lo - nb - 1, npx = Lo - nbx - 1;
    const IfaceCounts ic = iface_counts((uint32_t)Lo, (uint32_t)nbx, (uint32_t)nb);
    a.if_c0 = ic.c0;
    a.if_c01 = ic.c01;
    a.if_tot = ic.total;
    if (io.slots && (size_t)8 * ic.total * sizeof(T) > io.slots_bytes) {
        // slot code * total + t for the 8 side codes: more than the array holds
        set_error("interface partial sums need " + std::to_string((size_t)8 * ic.total * sizeof(T)) +
                  " bytes, more than the " + std::to_string(io.slots_bytes) + " of the scratch array");
        return FEM_ERR_WORKSPACE;
    }
    launch_p<KIND, T>(m.p, L.B, kvar, a, L.nbricks, s);
    FixGeom fg;
    fg.cnt0 = ic.c0;
    fg.cnt01 = ic.c01;
    fg.total = ic.total;
    fg.nbx = (uint32_t)nbx;
    fg.L = make_div((uint32_t)Lo);
    fg.LL = make_div((uint32_t)(Lo * Lo));
    fg.npx = make_div((uint32_t)std::max<int64_t>(npx, 1));
    fg.npxL = make_div((uint32_t)std::max<int64_t>(npx * Lo, 1));
    fg.npnpx = make_div((uint32_t)std::max<int64_t>(np * npx, 1));
    launch_fix<T>(po, L.B, a, fg, s);
    return check_launch("scatter kernel");
}

}  // namespace

template <typename T>
fem_status run_scatter(const fem_mesh& m, int level, int kind, bool kvar, const ScatterIO<T>& io, hipStream_t s) {
    switch (kind) {
        case K_APPLY: return run_kind<K_APPLY, T>(m, level, kvar, io, s);
        case K_DIAG: return run_kind<K_DIAG, T>(m, level, kvar, io, s);
        case K_MASS: return run_kind<K_MASS, T>(m, level, false, io, s);
        case K_GRAD:
            if constexpr (sizeof(T) == 8) return run_kind<K_GRAD, T>(m, level, false, io, s);
            break;
        default: break;
    }
    set_error("unsupported scatter kind");
    return FEM_ERR_UNSUPPORTED;
}

template fem_status run_scatter<double>(const fem_mesh&, int, int, bool, const ScatterIO<double>&, hipStream_t);
template fem_status run_scatter<float>(const fem_mesh&, int, int, bool, const ScatterIO<float>&, hipStream_t);

fem_status check_launch(const char* what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string(what) + ": " + hipGetErrorString(e));
        return FEM_ERR_HIP;
    }
    return FEM_OK;
}

}  // namespace fem
