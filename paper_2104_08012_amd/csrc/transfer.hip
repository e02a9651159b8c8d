// Multigrid transfers on the dof lattice.
//
// Prolongation x_f += P x_c (interpolation between the nested spaces).  Large P1/P2 levels: one
// thread per coarse cube, consecutive threads along x; the thread loads the (p+1)^3 coarse values
// of its cube and adds to every fine dof at local position r in [0, 2p)^3 of the cube (and r = 2p
// on the far faces of the last cube along an axis) the interpolant there: the coarse nodes of the
// tetrahedron holding the point weighted by their basis functions' values (a compile-time table of
// exact rational weights, rounded once).  Small levels and P3: one thread per fine dof reading the
// same table from memory (transfer.cpp).
// Restriction r_c = P^T r_f with boundary rows zero.  P1 and large P2 levels: one thread per
// coarse dof, the threads of a launch row (blockIdx.y) all of one residue class modulo p, so each
// wave runs its class's compile-time stencil (fine offsets d in [-2p, 2p]^3 with P[2J + d][J] != 0)
// over r_f at 2J + d; coarse dofs at least p from the boundary skip the bounds checks.  P3 (27
// classes, up to 427 stencil entries) and small P2 levels: 8 lanes per coarse dof walk the class's
// stencil from the table and add their partial sums by a fixed butterfly.
// Both write every output once in a fixed order of terms: deterministic, one launch each, no
// interface pass.
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

// Small levels (and P3): one thread per fine dof.  The dof's coarse cube and local position r in
// [0, 2p]^3 follow from its lattice point (the last cube along an axis takes the far face); the
// position's table row (transfer.cpp) lists the coarse nodes of the tetrahedron holding it and
// their weights, padded with zero weights, so every lane runs the same nloc steps.
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

// Interpolation weights of the fine positions r in [0, 2p]^3 of a coarse cube: the point lies in
// the path tetrahedron whose axis order sorts r decreasingly, with barycentric coordinates
// lambda = (2p - r_s0, r_s0 - r_s1, r_s1 - r_s2, r_s2) / (2p); the basis function of node m takes
// prod_w prod_{s < m_w} (p lambda_w - s) / (s + 1) there, an exact ratio of integers.  Nodes are
// listed in the element's node order, zero weights left out; node index a + (p+1)(b + (p+1)c)
// of the node's offset (a, b, c) in the cube.
template <int P>
struct ProlongTab {
    static constexpr int S = 2 * P + 1, NPOS = S * S * S, NL = nloc_of(P), PC = P + 1;
    int cnt[NPOS];
    int node[NPOS][NL];
    double w[NPOS][NL];
    constexpr ProlongTab() : cnt{}, node{}, w{} {
        const NodeList<P> nodes{};
        for (int pos = 0; pos < NPOS; ++pos) {
            const int r[3] = {pos % S, (pos / S) % S, pos / (S * S)};
            int t = 0;
            for (int tt = 5; tt >= 0; --tt)
                if (r[perm_axis(tt, 0)] >= r[perm_axis(tt, 1)] && r[perm_axis(tt, 1)] >= r[perm_axis(tt, 2)]) t = tt;
            const int s0 = perm_axis(t, 0), s1 = perm_axis(t, 1), s2 = perm_axis(t, 2);
            const int k[4] = {2 * P - r[s0], r[s0] - r[s1], r[s1] - r[s2], r[s2]};
            int V[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {1, 1, 1}};
            V[1][s0] = 1;
            V[2][s0] = 1;
            V[2][s1] = 1;
            int e = 0;
            for (int i = 0; i < NL; ++i) {
                long long num = 1, den = 1;
                for (int v = 0; v < 4; ++v)
                    for (int s = 0; s < nodes.m[i][v]; ++s) {
                        num *= (k[v] - 2 * s);
                        den *= 2 * (s + 1);
                    }
                if (num == 0) continue;
                int a[3] = {0, 0, 0};
                for (int v = 0; v < 4; ++v)
                    for (int d = 0; d < 3; ++d) a[d] += nodes.m[i][v] * V[v][d];
                node[pos][e] = a[0] + PC * (a[1] + PC * a[2]);
                w[pos][e] = (double)num / (double)den;
                ++e;
            }
            cnt[pos] = e;
        }
    }
};

template <int P, typename T>
__global__ void __launch_bounds__(256) k_prolong_cube(TArgs<T> a) {
    constexpr int S2 = 2 * P, PC = P + 1;
    constexpr ProlongTab<P> PT{};
    const uint32_t nc = a.nc, q = blockIdx.x * 256u + threadIdx.x;
    if (q >= nc * nc * nc) return;
    const uint32_t cx = q % nc, cy = (q / nc) % nc, cz = q / (nc * nc);
    const uint32_t Lc = a.Lc, Lf = a.Lf;
    T xc[PC * PC * PC];
    const uint32_t cb = P * cx + Lc * (P * cy + Lc * (P * cz));
#pragma unroll
    for (int c = 0; c < PC; ++c)
#pragma unroll
        for (int b = 0; b < PC; ++b)
#pragma unroll
            for (int a0 = 0; a0 < PC; ++a0)
                xc[a0 + PC * (b + PC * c)] = ldg(a.in, cb + (uint32_t)a0 + Lc * ((uint32_t)b + Lc * (uint32_t)c));
    // far faces: the last cube along an axis also takes r = 2p
    const int ex = cx == nc - 1 ? S2 : S2 - 1, ey = cy == nc - 1 ? S2 : S2 - 1, ez = cz == nc - 1 ? S2 : S2 - 1;
    const uint32_t fb = S2 * cx + Lf * (S2 * cy + Lf * (S2 * cz));
#pragma unroll
    for (int rz = 0; rz <= S2; ++rz)
#pragma unroll
        for (int ry = 0; ry <= S2; ++ry)
#pragma unroll
            for (int rx = 0; rx <= S2; ++rx) {
                if (rx > ex || ry > ey || rz > ez) continue;
                constexpr int S = S2 + 1;
                const int pos = rx + S * (ry + S * rz);
                T acc = T(0);
#pragma unroll
                for (int e = 0; e < PT.cnt[pos]; ++e) acc += T(PT.w[pos][e]) * xc[PT.node[pos][e]];
                const uint32_t f = fb + (uint32_t)rx + Lf * ((uint32_t)ry + Lf * (uint32_t)rz);
                stg(a.out, f, ldg(a.out, f) + acc);
            }
}

// Restriction stencils of the residue classes of a coarse node J modulo p (P1, P2): the fine
// offsets d in [-2p, 2p]^3 (z, then y, then x) with P[2J + d][J] != 0 and those weights, read
// from the interpolation table at an interior representative J = rho + 3p of the class.
template <int P>
struct RestrictTab {
    static constexpr int NCL = P * P * P, MAXE = P == 1 ? 15 : 125, S = 2 * P + 1, PC = P + 1;
    static_assert(P <= 2, "compile-time restriction stencils for P1 and P2");
    int cnt[NCL];
    int d[NCL][MAXE][3];
    double w[NCL][MAXE];
    constexpr RestrictTab() : cnt{}, d{}, w{} {
        const ProlongTab<P> PT{};
        for (int cls = 0; cls < NCL; ++cls) {
            const int J[3] = {cls % P + 3 * P, (cls / P) % P + 3 * P, cls / (P * P) + 3 * P};
            int e = 0;
            for (int dz = -2 * P; dz <= 2 * P; ++dz)
                for (int dy = -2 * P; dy <= 2 * P; ++dy)
                    for (int dx = -2 * P; dx <= 2 * P; ++dx) {
                        const int F[3] = {2 * J[0] + dx, 2 * J[1] + dy, 2 * J[2] + dz};
                        int c[3] = {0, 0, 0}, r[3] = {0, 0, 0};
                        for (int k = 0; k < 3; ++k) {
                            c[k] = F[k] / (2 * P);
                            r[k] = F[k] - 2 * P * c[k];
                        }
                        const int pos = r[0] + S * (r[1] + S * r[2]);
                        double wt = 0.0;
                        for (int q = 0; q < PT.cnt[pos]; ++q) {
                            const int nd = PT.node[pos][q];
                            const int a0 = nd % PC, a1 = (nd / PC) % PC, a2 = nd / (PC * PC);
                            if (P * c[0] + a0 == J[0] && P * c[1] + a1 == J[1] && P * c[2] + a2 == J[2]) wt = PT.w[pos][q];
                        }
                        if (wt == 0.0 || e >= MAXE) continue;
                        d[cls][e][0] = dx;
                        d[cls][e][1] = dy;
                        d[cls][e][2] = dz;
                        w[cls][e] = wt;
                        ++e;
                    }
            cnt[cls] = e;
        }
    }
};
static_assert(RestrictTab<1>{}.cnt[0] == 15, "P1 restriction stencil: 15 fine points");
static_assert(RestrictTab<2>{}.cnt[0] == 125 && RestrictTab<2>{}.cnt[1] == 27 && RestrictTab<2>{}.cnt[3] == 19,
              "P2 restriction stencils: 125 (vertex class), 27 and 19 fine points");

template <int P, int CLS, typename T>
__device__ __forceinline__ void restrict_class(const TArgs<T>& a, uint32_t i) {
    constexpr RestrictTab<P> RT{};
    constexpr int NE = RT.cnt[CLS];
    constexpr uint32_t rho0 = CLS % P, rho1 = (CLS / P) % P, rho2 = CLS / (P * P);
    const uint32_t nx = rho0 == 0 ? a.nc + 1 : a.nc, ny = rho1 == 0 ? a.nc + 1 : a.nc, nz = rho2 == 0 ? a.nc + 1 : a.nc;
    if (i >= nx * ny * nz) return;
    const uint32_t ix = i % nx, iy = (i / nx) % ny, iz = i / (nx * ny);
    const uint32_t JX = rho0 + P * ix, JY = rho1 + P * iy, JZ = rho2 + P * iz;
    const uint32_t Lc = a.Lc, j = JX + Lc * (JY + Lc * JZ);
    const bool bnd = JX == 0 || JY == 0 || JZ == 0 || JX == Lc - 1 || JY == Lc - 1 || JZ == Lc - 1;
    T acc = T(0);
    if (!bnd) {
        const int Lf = (int)a.Lf;
        const int FX = 2 * (int)JX, FY = 2 * (int)JY, FZ = 2 * (int)JZ;
        const bool inner = JX >= (uint32_t)P && JY >= (uint32_t)P && JZ >= (uint32_t)P && JX + P < Lc &&
                           JY + P < Lc && JZ + P < Lc;
        if (inner) {
            const uint32_t c = (uint32_t)FX + (uint32_t)Lf * ((uint32_t)FY + (uint32_t)Lf * (uint32_t)FZ);
#pragma unroll
            for (int e = 0; e < NE; ++e)
                acc += T(RT.w[CLS][e]) * ldg(a.in, (uint32_t)((int)c + RT.d[CLS][e][0] + Lf * (RT.d[CLS][e][1] + Lf * RT.d[CLS][e][2])));
        } else {
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                const int x = FX + RT.d[CLS][e][0], y = FY + RT.d[CLS][e][1], z = FZ + RT.d[CLS][e][2];
                if (x >= 0 && y >= 0 && z >= 0 && x < Lf && y < Lf && z < Lf)
                    acc += T(RT.w[CLS][e]) * ldg(a.in, (uint32_t)x + (uint32_t)Lf * ((uint32_t)y + (uint32_t)Lf * (uint32_t)z));
            }
        }
    }
    a.out[j] = acc;
}

template <int P, typename T, int... CLS>
__device__ __forceinline__ void restrict_dispatch(const TArgs<T>& a, uint32_t i, int cls, std::integer_sequence<int, CLS...>) {
    ((cls == CLS ? restrict_class<P, CLS, T>(a, i) : void()), ...);
}

// one thread per coarse dof; launch row blockIdx.y = the residue class
template <int P, typename T>
__global__ void __launch_bounds__(256) k_restrict_class(TArgs<T> a) {
    const int cls = __builtin_amdgcn_readfirstlane((int)blockIdx.y);
    restrict_dispatch<P, T>(a, blockIdx.x * 256u + threadIdx.x, cls, std::make_integer_sequence<int, P * P * P>{});
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

// coarse levels of at least this many cubes per direction prolong one thread per coarse cube, and
// (P2) restrict one thread per coarse dof; smaller ones, where a kernel's time is one thread's
// chain of loads, take the table kernels (8 lanes per coarse dof for the restriction)
constexpr uint32_t kProlongCubeMinN = 32;
constexpr uint32_t kRestrictClassMinN = 32;

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
    // one thread per coarse cube once there are enough cubes to fill the GPU (a thread's 8 (P1)
    // or 64 (P2) fine points are a serial chain that small levels cannot hide); else per fine dof
    if (m.p <= 2 && a.nc >= kProlongCubeMinN) {
        const dim3 grid((a.nc * a.nc * a.nc + 255) / 256);
        if (m.p == 1) hipLaunchKernelGGL((k_prolong_cube<1, T>), grid, dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_prolong_cube<2, T>), grid, dim3(256), 0, s, a);
        return check_launch("prolongation kernel");
    }
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
    if (m.p == 1) hipLaunchKernelGGL((k_restrict_class<1, T>), dim3((n1 * n1 * n1 + 255) / 256, 1), dim3(256), 0, s, a);
    else if (m.p == 2 && a.nc >= kRestrictClassMinN)
        hipLaunchKernelGGL((k_restrict_class<2, T>), dim3((n1 * n1 * n1 + 255) / 256, 8), dim3(256), 0, s, a);
    else if (m.p == 2) hipLaunchKernelGGL((k_restrict_lattice<2, T>), dim3((8 * n1 * n1 * n1 + 255) / 256, 8), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_restrict_lattice<3, T>), dim3((8 * n1 * n1 * n1 + 255) / 256, 27), dim3(256), 0, s, a);
    return check_launch("restriction kernel");
}

template fem_status run_prolong<double>(const fem_mesh&, int, const double*, double*, hipStream_t);
template fem_status run_prolong<float>(const fem_mesh&, int, const float*, float*, hipStream_t);
template fem_status run_restrict<double>(const fem_mesh&, int, const double*, double*, hipStream_t);
template fem_status run_restrict<float>(const fem_mesh&, int, const float*, float*, hipStream_t);

}  // namespace fem
