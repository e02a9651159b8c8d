// Additive vertex-star patch preconditioner for P2 and P3 (Section 2, Listing 2: the multigrid
// smoother is preconditioned by the patch preconditioner with star patches around the mesh
// vertices, combined additively):
//     z = sum_v R_v^T A_v^{-1} R_v r      on interior dofs,   z_B = r_B,
// R_v the restriction to the interior dofs of the star of vertex v, A_v = R_v A R_v^T.  The star
// slots (15 dofs for P2, 65 for P3) and the cells around a vertex are the tables of star.hpp.
// Dofs outside the lattice or on the boundary are left out (zero rows and columns of the stored
// inverse).
//
// Setup (one 64-lane workgroup per vertex, the star matrix in LDS): A_v is summed from the
// element matrices of the 24 cells around v (the only cells coupling two star dofs), restricted
// to their star nodes, one cell after the other in a fixed order, with the quadrature rule of
// the P1-coefficient stiffness (exact for k = 1 too), the cell's geometric factor G and the
// vertex values of k; then inverted by Gauss-Jordan elimination in LDS in FP64 (A_v is symmetric
// positive definite, so no pivoting) and stored as its packed lower triangle (120 entries per
// vertex for P2, 2145 for P3) in blocks of 64 vertices: entry e of vertex v at
// ((v / 64) NE + e) 64 + v % 64 (NE entries per vertex), so the 64 lanes of a wave read 512
// contiguous bytes per entry and a wave's whole stream is one contiguous region.
// Apply: a per-star product of every star's inverse with the gathered residual (P2: one thread
// per vertex, all in registers; P3: one thread per vertex with the residual and the symmetric
// half of the products in LDS, rows in blocks held in registers), storing the star results per
// vertex in the same blocked layout; then k_patch_combine sums, for every dof, the results of the one to three stars
// that contain it in increasing vertex order (a deterministic gather, no atomics).
#include <hip/hip_runtime.h>

#include "ops.hpp"
#include "star.hpp"
#include "tabulate.hpp"

namespace fem {

namespace {

template <int P>
__device__ constexpr StarTab<P> kStarTab{};
template <int P>
__device__ constexpr StiffTab<P, true> kStarRule{};

struct PatchGeom {
    int n, B, nb, NC;
    uint32_t C, NV, L;
};

// blocked per-vertex layout of the packed inverses and star results (NE entries per vertex)
__device__ __forceinline__ uint32_t pblock(uint32_t v, uint32_t NE) { return (v >> 6) * NE * 64u + (v & 63u); }

// Lattice point of star slot s of vertex (vi, vj, vk) and whether it is an interior dof.
template <int P>
__device__ inline bool star_point(int s, int vi, int vj, int vk, int Lm, uint32_t L, uint32_t& idx) {
    const int X = P * vi + kStarTab<P>.off[s][0], Y = P * vj + kStarTab<P>.off[s][1],
              Z = P * vk + kStarTab<P>.off[s][2];
    idx = (uint32_t)X + L * ((uint32_t)Y + L * (uint32_t)Z);
    return X > 0 && Y > 0 && Z > 0 && X < Lm && Y < Lm && Z < Lm;
}

template <int P, typename T>
__global__ void __launch_bounds__(64) k_star_setup(PatchGeom g, const double* __restrict__ G,
                                                   const double* __restrict__ kv, T* __restrict__ inv) {
    constexpr int NS = StarTab<P>::NS, LD = NS + 1, NCN = StarTab<P>::NCN, NQ = StiffTab<P, true>::NQ;
    __shared__ double A[NS * LD];
    __shared__ double colp[NS];
    __shared__ double gd[NQ * NCN * 3];
    const auto& st = kStarTab<P>;
    const auto& tab = kStarRule<P>;
    const uint32_t v = blockIdx.x;
    const int lane = threadIdx.x;
    const int n = g.n, N1 = n + 1, Lm = P * n;
    const int vi = (int)(v % N1), vj = (int)((v / N1) % N1), vk = (int)(v / (N1 * N1));
    for (int e = lane; e < NS * LD; e += 64) A[e] = 0.0;
    __syncthreads();
    const int B3 = g.B * g.B * g.B;
    for (int o = 0; o < 8; ++o) {
        const int cx = vi - (o & 1), cy = vj - ((o >> 1) & 1), cz = vk - (o >> 2);
        if (cx < 0 || cy < 0 || cz < 0 || cx >= n || cy >= n || cz >= n) continue;
        const int brick = cx / g.B + g.nb * (cy / g.B + g.nb * (cz / g.B));
        const int cl = cx % g.B + g.B * (cy % g.B + g.B * (cz % g.B));
        for (int t = 0; t < 6; ++t) {
            if (st.iv[o][t] < 0) continue;
            const uint32_t c = (uint32_t)brick * g.NC + t * B3 + cl;
            const double G00v = G[c], G11v = G[g.C + c], G22v = G[2 * g.C + c], G01v = G[3 * g.C + c],
                         G02v = G[4 * g.C + c], G12v = G[5 * g.C + c];
            const int s0 = perm_axis(t, 0), s1 = perm_axis(t, 1);
            double kc[4];
            for (int w = 0; w < 4; ++w) {
                const int dx = (w >= 1 && s0 == 0) || (w >= 2 && s1 == 0) || w == 3;
                const int dy = (w >= 1 && s0 == 1) || (w >= 2 && s1 == 1) || w == 3;
                const int dz = (w >= 1 && s0 == 2) || (w >= 2 && s1 == 2) || w == 3;
                const uint32_t vid = (uint32_t)(cx + dx) + N1 * ((uint32_t)(cy + dy) + N1 * (uint32_t)(cz + dz));
                kc[w] = kv ? kv[vid] : 1.0;
            }
            // w_q k(x_q) G grad(phi_a)(x_q) for the cell's star nodes a
            for (int e = lane; e < NQ * NCN; e += 64) {
                const int q = e / NCN, a = e % NCN, i = st.cn[o][t][a];
                const double kq = tab.lam[q][0] * kc[0] + tab.lam[q][1] * kc[1] + tab.lam[q][2] * kc[2] +
                                  tab.lam[q][3] * kc[3];
                const double wk = tab.w[q] * kq;
                const double d0 = tab.D[q][0][i], d1 = tab.D[q][1][i], d2 = tab.D[q][2][i];
                gd[3 * e] = wk * (G00v * d0 + G01v * d1 + G02v * d2);
                gd[3 * e + 1] = wk * (G01v * d0 + G11v * d1 + G12v * d2);
                gd[3 * e + 2] = wk * (G02v * d0 + G12v * d1 + G22v * d2);
            }
            __syncthreads();
            // the cell's star block; its (slot a, slot b) pairs are distinct, so no two lanes add
            // to one entry, and the cells are summed one after the other in a fixed order
            for (int e = lane; e < NCN * NCN; e += 64) {
                const int a = e / NCN, b = e % NCN, j = st.cn[o][t][b];
                double sum = 0.0;
                for (int q = 0; q < NQ; ++q) {
                    const double* u = &gd[3 * (q * NCN + a)];
                    sum += u[0] * tab.D[q][0][j] + u[1] * tab.D[q][1][j] + u[2] * tab.D[q][2][j];
                }
                A[st.cs[o][t][a] * LD + st.cs[o][t][b]] += sum;
            }
            __syncthreads();
        }
    }
    // star dofs outside the lattice or on the boundary: identity rows and columns, zeroed after
    for (int e = lane; e < NS * NS; e += 64) {
        const int a = e / NS, b = e % NS;
        uint32_t ia, ib;
        const bool la = star_point<P>(a, vi, vj, vk, Lm, g.L, ia), lb = star_point<P>(b, vi, vj, vk, Lm, g.L, ib);
        if (!la || !lb) A[a * LD + b] = (a == b) ? 1.0 : 0.0;
    }
    __syncthreads();
    // in-place Gauss-Jordan inverse: for each pivot p, scale row p, then eliminate column p from
    // every other row using a copy of the column taken before the row was scaled
    for (int p = 0; p < NS; ++p) {
        for (int a = lane; a < NS; a += 64) colp[a] = A[a * LD + p];
        __syncthreads();
        const double piv = 1.0 / colp[p];
        for (int b = lane; b < NS; b += 64) A[p * LD + b] = (b == p) ? piv : A[p * LD + b] * piv;
        __syncthreads();
        for (int e = lane; e < NS * NS; e += 64) {
            const int a = e / NS, b = e % NS;
            if (a == p) continue;
            A[a * LD + b] = (b == p) ? -colp[a] * piv : A[a * LD + b] - colp[a] * A[p * LD + b];
        }
        __syncthreads();
    }
    for (int e = lane; e < NS * NS; e += 64) {
        const int a = e / NS, b = e % NS;
        if (b > a) continue;
        uint32_t ia, ib;
        const bool live = star_point<P>(a, vi, vj, vk, Lm, g.L, ia) && star_point<P>(b, vi, vj, vk, Lm, g.L, ib);
        const double val = live ? 0.5 * (A[a * LD + b] + A[b * LD + a]) : 0.0;
        inv[pblock(v, StarTab<P>::NP) + (uint32_t)(a * (a + 1) / 2 + b) * 64u] = (T)val;
    }
}

// P2: one thread per vertex, the 15 residual values and results in registers.
template <typename T>
__global__ void __launch_bounds__(256) k_patch_local2(PatchGeom g, const T* __restrict__ inv, const T* __restrict__ r,
                                                      T* __restrict__ u) {
    constexpr int NS = StarTab<2>::NS;
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= g.NV) return;
    const uint32_t ib = pblock(v, StarTab<2>::NP), ub = pblock(v, NS);
    const int n = g.n, N1 = n + 1, Lm = 2 * n;
    const int vi = (int)(v % N1), vj = (int)((v / N1) % N1), vk = (int)(v / (N1 * N1));
    T rs[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        uint32_t idx;
        rs[s] = star_point<2>(s, vi, vj, vk, Lm, g.L, idx) ? r[idx] : T(0);
    }
    T us[NS];
#pragma unroll
    for (int a = 0; a < NS; ++a) us[a] = T(0);
#pragma unroll
    for (int a = 0; a < NS; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            const T m = inv[ib + (uint32_t)(a * (a + 1) / 2 + b) * 64u];
            us[a] += m * rs[b];
            if (b != a) us[b] += m * rs[a];
        }
#pragma unroll
    for (int a = 0; a < NS; ++a) u[ub + (uint32_t)a * 64u] = us[a];
}

// P3: one thread per vertex (64 per workgroup).  The 65 residual values and the symmetric half of
// the products live in LDS (one column per lane); the packed rows are taken in blocks of RB
// (16 rows in FP64, 24 in FP32: each column b of a block issues RB independent coalesced loads,
// which is what keeps enough bytes in flight at two workgroups per CU) whose results stay in
// registers: for row a of the block and b < a the entry m_ab adds
// m_ab r_b to row a and m_ab r_a to row b (an LDS accumulation); the block's own lower triangle
// is unrolled.  Row a's result is complete once the later blocks have added their column-a terms.
template <typename T>
__global__ void __launch_bounds__(64) k_patch_local3(PatchGeom g, const T* __restrict__ inv, const T* __restrict__ r,
                                                     T* __restrict__ u) {
    constexpr int NS = StarTab<3>::NS, RB = sizeof(T) == 8 ? 16 : 24;   // the most rows without spills
    __shared__ T rs[NS][64];
    __shared__ T us[NS][64];
    const int lane = threadIdx.x;
    const uint32_t v = blockIdx.x * 64 + lane;
    const bool valid = v < g.NV;
    const uint32_t vv = valid ? v : 0;
    const uint32_t ib = pblock(v, StarTab<3>::NP), ub = pblock(v, NS);
    const int n = g.n, N1 = n + 1, Lm = 3 * n;
    const int vi = (int)(vv % N1), vj = (int)((vv / N1) % N1), vk = (int)(vv / (N1 * N1));
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        uint32_t idx;
        const bool live = star_point<3>(s, vi, vj, vk, Lm, g.L, idx);
        rs[s][lane] = (valid && live) ? r[idx] : T(0);
    }
    // each lane reads and writes only its own column of rs and us: no barrier is needed
#pragma unroll 1
    for (int a0 = 0; a0 < NS; a0 += RB) {
        const int nr = (NS - a0) < RB ? (NS - a0) : RB;
        T acc[RB], ra[RB];
        uint32_t row[RB];   // packed index of (a0 + j, 0)
#pragma unroll
        for (int j = 0; j < RB; ++j) {
            acc[j] = T(0);
            ra[j] = j < nr ? rs[a0 + j][lane] : T(0);
            row[j] = (uint32_t)((a0 + j) * (a0 + j + 1) / 2);
        }
#pragma unroll 4
        for (int b = 0; b < a0; ++b) {
            const T rb = rs[b][lane];
            T sym = T(0);
#pragma unroll
            for (int j = 0; j < RB; ++j) {
                const T m = (valid && j < nr) ? inv[ib + (row[j] + (uint32_t)b) * 64u] : T(0);
                acc[j] += m * rb;
                sym += m * ra[j];
            }
            us[b][lane] += sym;
        }
#pragma unroll
        for (int j = 0; j < RB; ++j)
#pragma unroll
            for (int jb = 0; jb <= j; ++jb) {
                const T m = (valid && j < nr) ? inv[ib + (row[j] + (uint32_t)(a0 + jb)) * 64u] : T(0);
                acc[j] += m * ra[jb];
                if (jb != j) acc[jb] += m * ra[j];
            }
#pragma unroll
        for (int j = 0; j < RB; ++j)
            if (j < nr) us[a0 + j][lane] = acc[j];
    }
    if (!valid) return;
#pragma unroll
    for (int a = 0; a < NS; ++a) u[ub + (uint32_t)a * 64u] = us[a][lane];
}

// z at every dof: the star results of the stars holding it (1 for a vertex, 2 for an edge node,
// 3 for a P3 face node), added in increasing vertex order; boundary dofs pass r through.
template <int P, typename T>
__global__ void __launch_bounds__(256) k_patch_combine(PatchGeom g, const T* __restrict__ u, const T* __restrict__ r,
                                                       T* __restrict__ z) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t L = g.L, N = L * L * L;
    if (i >= N) return;
    const uint32_t X = i % L, Y = (i / L) % L, Z = i / (L * L);
    if (X == 0 || Y == 0 || Z == 0 || X == L - 1 || Y == L - 1 || Z == L - 1) {
        z[i] = r[i];
        return;
    }
    const uint32_t N1 = (uint32_t)g.n + 1;
    const uint32_t cx = X / P, cy = Y / P, cz = Z / P, rx = X % P, ry = Y % P, rz = Z % P;
    const uint32_t base = cx + N1 * (cy + N1 * cz);
    const auto& st = kStarTab<P>;
    const int cnt = st.rn[rx][ry][rz];
    T acc = T(0);
    for (int k = 0; k < cnt; ++k) {
        const int bits = st.rv[rx][ry][rz][k];
        const uint32_t vid = base + (uint32_t)(bits & 1) + N1 * ((uint32_t)((bits >> 1) & 1) + N1 * (uint32_t)(bits >> 2));
        const T uk = u[pblock(vid, StarTab<P>::NS) + (uint32_t)st.rs[rx][ry][rz][k] * 64u];
        acc = k == 0 ? uk : acc + uk;
    }
    z[i] = acc;
}

PatchGeom patch_geom(const HostLevel& H) {
    PatchGeom g;
    g.n = H.n;
    g.B = H.B;
    g.nb = H.nb;
    g.NC = H.NC;
    g.C = (uint32_t)H.C;
    g.NV = (uint32_t)H.NV;
    g.L = (uint32_t)H.L;
    return g;
}

int star_size(int p) { return p == 2 ? StarTab<2>::NS : p == 3 ? StarTab<3>::NS : 0; }
int64_t padded_vertices(const HostLevel& H) { return (H.NV + 63) / 64 * 64; }
int star_packed(int p) { return p == 2 ? StarTab<2>::NP : p == 3 ? StarTab<3>::NP : 0; }

}  // namespace

bool patch_supported(const HostLevel& H, std::string& why) {
    if (H.p != 2 && H.p != 3) {
        why = "star patches are built for degrees 2 and 3 (for degree 1 every star is one dof: Jacobi)";
        return false;
    }
    // packed entry e of vertex v is element ((v / 64) NE + e) 64 + v % 64 (32-bit), over the
    // vertex count rounded up to a multiple of 64
    if ((uint64_t)(star_packed(H.p) + star_size(H.p)) * (uint64_t)padded_vertices(H) >= ((uint64_t)1 << 32)) {
        why = "level has too many vertices for the 32-bit packed star index (" + std::to_string(star_packed(H.p)) +
              " entries per vertex)";
        return false;
    }
    return true;
}

size_t patch_bytes(const HostLevel& H, size_t ts) {
    const size_t nv = padded_vertices(H);
    return align256((size_t)star_packed(H.p) * nv * ts) + align256((size_t)star_size(H.p) * nv * ts);
}

template <typename T>
fem_status patch_setup(const fem_mesh& m, int level, const double* k, void* buf, hipStream_t s) {
    const HostLevel& H = m.lev[level];
    const PatchGeom g = patch_geom(H);
    T* inv = reinterpret_cast<T*>(buf);
    if (H.p == 2)
        hipLaunchKernelGGL((k_star_setup<2, T>), dim3(g.NV), dim3(64), 0, s, g, dptr<double>(m, H.d_G64), k, inv);
    else
        hipLaunchKernelGGL((k_star_setup<3, T>), dim3(g.NV), dim3(64), 0, s, g, dptr<double>(m, H.d_G64), k, inv);
    return check_launch("fem_patch_setup");
}

template <typename T>
fem_status patch_apply(const fem_mesh& m, int level, void* buf, const T* r, T* z, hipStream_t s) {
    const HostLevel& H = m.lev[level];
    const PatchGeom g = patch_geom(H);
    const T* inv = reinterpret_cast<const T*>(buf);
    T* u = reinterpret_cast<T*>(reinterpret_cast<char*>(buf) +
                                align256((size_t)star_packed(H.p) * padded_vertices(H) * sizeof(T)));
    const unsigned gc = (unsigned)((H.N + 255) / 256);
    if (H.p == 2) {
        hipLaunchKernelGGL((k_patch_local2<T>), dim3((g.NV + 255) / 256), dim3(256), 0, s, g, inv, r, u);
        hipLaunchKernelGGL((k_patch_combine<2, T>), dim3(gc), dim3(256), 0, s, g, (const T*)u, r, z);
    } else {
        hipLaunchKernelGGL((k_patch_local3<T>), dim3((g.NV + 63) / 64), dim3(64), 0, s, g, inv, r, u);
        hipLaunchKernelGGL((k_patch_combine<3, T>), dim3(gc), dim3(256), 0, s, g, (const T*)u, r, z);
    }
    return check_launch("fem_apply_patch");
}

template fem_status patch_setup<double>(const fem_mesh&, int, const double*, void*, hipStream_t);
template fem_status patch_setup<float>(const fem_mesh&, int, const double*, void*, hipStream_t);
template fem_status patch_apply<double>(const fem_mesh&, int, void*, const double*, double*, hipStream_t);
template fem_status patch_apply<float>(const fem_mesh&, int, void*, const float*, float*, hipStream_t);

}  // namespace fem
