// Multigrid transfers on the dof lattice (tables: transfer.cpp).
//
// Prolongation x_f += P x_c: one thread per fine dof.  The dof's coarse cube and local position r
// in [0, 2p]^3 follow from its lattice point (the last cube along an axis takes the far face);
// the position's table row lists the coarse nodes of the tetrahedron holding it and their
// weights, padded with zero weights, so every lane runs the same nloc steps.
// Restriction r_c = P^T r_f with boundary rows zero: 8 lanes per coarse dof, the threads of a
// launch row (blockIdx.y) all of one residue class modulo p, so a wave walks one shared stencil
// and gathers r_f at 2 J + d (linear offsets per level; coarse dofs at least p from the boundary
// skip the bounds checks); boundary rows are zero.
// Both write every output once in a fixed order of terms: deterministic, one launch each, no
// interface pass.  Consecutive threads take consecutive lattice points (coalesced x_f, and r_c
// at stride p).
#include <hip/hip_runtime.h>

#include "ops.hpp"
#include "scatter.hpp"

namespace fem {

namespace {

template <typename T>
struct TArgs {
    uint32_t Nf, Lf, Lc, nc, ncl_count[3];
    Div Lfd, LLfd;
    const T* in;
    T* out;
    const int32_t* pt_off;
    const T* pt_w;
    const int32_t* rs_start;
    const int32_t* rs_off;
    const int32_t* rs_lin;
    const T* rs_w;
};

template <int P, typename T>
__global__ void __launch_bounds__(256) k_prolong_lattice(TArgs<T> a) {
    constexpr int S2 = 2 * P, S = S2 + 1, NE = nloc_of(P);
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i >= a.Nf) return;
    const uint32_t K = udiv(i, a.LLfd), rem = i - K * a.LLfd.d, J = udiv(rem, a.Lfd), I = rem - J * a.Lf;
    const uint32_t ncm = a.nc - 1;
    const uint32_t cx = min(I / S2, ncm), cy = min(J / S2, ncm), cz = min(K / S2, ncm);
    const uint32_t rx = I - S2 * cx, ry = J - S2 * cy, rz = K - S2 * cz;
    const uint32_t pos = rx + S * (ry + S * rz);
    const uint32_t Lc = a.Lc;
    const uint32_t base = P * cx + Lc * (P * cy + Lc * (P * cz));
    T acc = T(0);
#pragma unroll
    for (int e = 0; e < NE; ++e) {
        const int o = a.pt_off[pos * NE + e];
        const T w = a.pt_w[pos * NE + e];
        const uint32_t idx = base + (uint32_t)(o & 255) + Lc * ((uint32_t)((o >> 8) & 255) + Lc * (uint32_t)(o >> 16));
        acc += w * ldg(a.in, idx);
    }
    a.out[i] += acc;
}

// 8 lanes per coarse dof, each summing every eighth stencil entry; the 8 partial sums are added
// by a fixed butterfly, so the result does not depend on scheduling.
template <int P, typename T>
__global__ void __launch_bounds__(256) k_restrict_lattice(TArgs<T> a) {
    constexpr int D = 4 * P + 1, G = 8;
    const int cls = blockIdx.y;
    const uint32_t rho[3] = {(uint32_t)(cls % P), (uint32_t)((cls / P) % P), (uint32_t)(cls / (P * P))};
    const uint32_t nx = rho[0] == 0 ? a.nc + 1 : a.nc, ny = rho[1] == 0 ? a.nc + 1 : a.nc,
                   nz = rho[2] == 0 ? a.nc + 1 : a.nc;
    const uint32_t gi = blockIdx.x * 256u + threadIdx.x, i = gi / G;
    const int part = (int)(gi % G);
    const bool valid = i < nx * ny * nz;
    const uint32_t ii = valid ? i : 0;
    const uint32_t ix = ii % nx, iy = (ii / nx) % ny, iz = ii / (nx * ny);
    const uint32_t JX = rho[0] + P * ix, JY = rho[1] + P * iy, JZ = rho[2] + P * iz;
    const uint32_t Lc = a.Lc, j = JX + Lc * (JY + Lc * JZ);
    const bool bnd = JX == 0 || JY == 0 || JZ == 0 || JX == Lc - 1 || JY == Lc - 1 || JZ == Lc - 1;
    T acc = T(0);
    if (valid && !bnd) {
        const int e0 = a.rs_start[cls] + part, e1 = a.rs_start[cls + 1];
        const int Lf = (int)a.Lf;
        const int FX = 2 * (int)JX - 2 * P, FY = 2 * (int)JY - 2 * P, FZ = 2 * (int)JZ - 2 * P;
        const bool inner = JX >= (uint32_t)P && JY >= (uint32_t)P && JZ >= (uint32_t)P && JX + P < Lc &&
                           JY + P < Lc && JZ + P < Lc;
        if (inner) {
            const uint32_t c = (uint32_t)(2 * (int)JX) + (uint32_t)Lf * ((uint32_t)(2 * (int)JY) + (uint32_t)Lf * (uint32_t)(2 * (int)JZ));
#pragma unroll 4
            for (int e = e0; e < e1; e += G) acc += a.rs_w[e] * ldg(a.in, (uint32_t)((int)c + a.rs_lin[e]));
        } else {
            for (int e = e0; e < e1; e += G) {
                const int o = a.rs_off[e];
                const int x = FX + o % D, y = FY + (o / D) % D, z = FZ + o / (D * D);
                if (x >= 0 && y >= 0 && z >= 0 && x < Lf && y < Lf && z < Lf)
                    acc += a.rs_w[e] * ldg(a.in, (uint32_t)x + (uint32_t)Lf * ((uint32_t)y + (uint32_t)Lf * (uint32_t)z));
            }
        }
    }
#pragma unroll
    for (int s = 1; s < G; s <<= 1) acc += __shfl_xor(acc, s, G);
    if (valid && part == 0) a.out[j] = acc;
}

template <typename T>
const T* wtab(const fem_mesh& m, size_t off64, size_t off32) {
    return reinterpret_cast<const T*>(m.dev + (sizeof(T) == 8 ? off64 : off32));
}

template <typename T>
TArgs<T> targs(const fem_mesh& m, int fine_level, const T* in, T* out) {
    const HostLevel& Lc = m.lev[fine_level - 1];
    const HostLevel& Lf = m.lev[fine_level];
    TArgs<T> a{};
    a.Nf = (uint32_t)Lf.N;
    a.Lf = (uint32_t)Lf.L;
    a.Lc = (uint32_t)Lc.L;
    a.nc = (uint32_t)Lc.n;
    a.Lfd = make_div((uint32_t)Lf.L);
    a.LLfd = make_div((uint32_t)(Lf.L * Lf.L));
    a.in = in;
    a.out = out;
    a.pt_off = dptr<int32_t>(m, m.d_pt_off);
    a.pt_w = wtab<T>(m, m.d_pt_w64, m.d_pt_w32);
    a.rs_start = dptr<int32_t>(m, m.d_rs_start);
    a.rs_off = dptr<int32_t>(m, m.d_rs_off);
    a.rs_lin = dptr<int32_t>(m, Lc.d_rs_lin);
    a.rs_w = wtab<T>(m, m.d_rs_w64, m.d_rs_w32);
    return a;
}

}  // namespace

template <typename T>
fem_status run_prolong(const fem_mesh& m, int fine_level, const T* xc, T* xf, hipStream_t s) {
    const TArgs<T> a = targs<T>(m, fine_level, xc, xf);
    const dim3 grid((a.Nf + 255) / 256);
    if (m.p == 1) hipLaunchKernelGGL((k_prolong_lattice<1, T>), grid, dim3(256), 0, s, a);
    else if (m.p == 2) hipLaunchKernelGGL((k_prolong_lattice<2, T>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_prolong_lattice<3, T>), grid, dim3(256), 0, s, a);
    return check_launch("prolongation kernel");
}

template <typename T>
fem_status run_restrict(const fem_mesh& m, int fine_level, const T* rf, T* rc, hipStream_t s) {
    const TArgs<T> a = targs<T>(m, fine_level, rf, rc);
    const uint32_t n1 = a.nc + 1;
    const dim3 grid((8 * n1 * n1 * n1 + 255) / 256, m.p * m.p * m.p);
    if (m.p == 1) hipLaunchKernelGGL((k_restrict_lattice<1, T>), grid, dim3(256), 0, s, a);
    else if (m.p == 2) hipLaunchKernelGGL((k_restrict_lattice<2, T>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_restrict_lattice<3, T>), grid, dim3(256), 0, s, a);
    return check_launch("restriction kernel");
}

template fem_status run_prolong<double>(const fem_mesh&, int, const double*, double*, hipStream_t);
template fem_status run_prolong<float>(const fem_mesh&, int, const float*, float*, hipStream_t);
template fem_status run_restrict<double>(const fem_mesh&, int, const double*, double*, hipStream_t);
template fem_status run_restrict<float>(const fem_mesh&, int, const float*, float*, hipStream_t);

}  // namespace fem
