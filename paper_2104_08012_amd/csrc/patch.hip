// Additive vertex-star patch preconditioner for P2 (Section 2, Listing 2: the multigrid smoother
// is preconditioned by the patch preconditioner with star patches around the mesh vertices,
// combined additively):
//     z = sum_v R_v^T A_v^{-1} R_v r      on interior dofs,   z_B = r_B,
// R_v the restriction to the interior dofs of the star of vertex v, A_v = R_v A R_v^T.
//
// Star of a vertex in the cube split.  The edges of the split are the lattice vectors with 0/1
// components (axes, the (1,1,0)-type face diagonals and the main diagonal), 7 per direction sign,
// so on the P2 lattice (spacing h/2) the star of vertex v (lattice point 2v) holds
//   s = 0:          the vertex dof 2v,
//   s = c (1..7):   the edge midpoint 2v + d(c),
//   s = 7 + c:      the edge midpoint 2v - d(c),          d(c) = (c & 1, (c >> 1) & 1, c >> 2).
// Dofs outside the lattice or on the boundary are left out (zero rows and columns of the stored
// inverse).  Every edge midpoint 2u + d lies in the stars of u (slot c) and u + d (slot 7 + c).
//
// Setup (one thread per vertex): A_v is summed from the element matrices of the cells around v
// (the only cells coupling two star dofs), restricted to their four star nodes, with the
// degree-3 rule of the P1-coefficient stiffness (exact for k = 1 too), the cell's geometric
// factor G and the vertex values of k; then inverted by Gauss-Jordan elimination in FP64 (A_v is
// symmetric positive definite, so no pivoting) and stored as its packed lower triangle, 120
// entries per vertex, structure of arrays.
// Apply: k_patch_local multiplies every star's inverse with the gathered residual and stores the
// 15 patch results per vertex; k_patch_combine sums, for every dof, the results of the one or two
// stars that contain it (a deterministic gather, no atomics).
#include <hip/hip_runtime.h>

#include "ops.hpp"
#include "tabulate.hpp"

namespace fem {

namespace {

constexpr int kStar = 15, kPacked = kStar * (kStar + 1) / 2;

struct PatchGeom {
    int n, B, nb, NC;
    uint32_t C, NV, L;
};

FEM_HD inline int star_slot(int ox, int oy, int oz) {
    if (ox == 0 && oy == 0 && oz == 0) return 0;
    if (ox >= 0 && oy >= 0 && oz >= 0) return ox + 2 * oy + 4 * oz;
    return 7 + (-ox) + 2 * (-oy) + 4 * (-oz);
}

__device__ inline int packed(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }

template <typename T>
__global__ void __launch_bounds__(64) k_patch_setup(PatchGeom g, const double* __restrict__ G,
                                                    const double* __restrict__ kv, T* __restrict__ inv) {
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= g.NV) return;
    const int n = g.n, N1 = n + 1;
    const int vi = (int)(v % N1), vj = (int)((v / N1) % N1), vk = (int)(v / (N1 * N1));
    constexpr StiffTab<2, true> tab{};
    constexpr NodeList<2> nodes{};
    constexpr int ea[6] = {0, 0, 0, 1, 1, 2}, eb[6] = {1, 2, 3, 2, 3, 3};
    double A[kStar][kStar];
    for (int a = 0; a < kStar; ++a)
        for (int b = 0; b < kStar; ++b) A[a][b] = 0.0;
    const int B3 = g.B * g.B * g.B;
    for (int o = 0; o < 8; ++o) {
        const int ox = o & 1, oy = (o >> 1) & 1, oz = o >> 2;
        const int cx = vi - ox, cy = vj - oy, cz = vk - oz;
        if (cx < 0 || cy < 0 || cz < 0 || cx >= n || cy >= n || cz >= n) continue;
        const int brick = cx / g.B + g.nb * (cy / g.B + g.nb * (cz / g.B));
        const int cl = cx % g.B + g.B * (cy % g.B + g.B * (cz % g.B));
        for (int t = 0; t < 6; ++t) {
            const int s0 = perm_axis(t, 0), s1 = perm_axis(t, 1);
            int V[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {1, 1, 1}};
            V[1][s0] = 1;
            V[2][s0] = 1;
            V[2][s1] = 1;
            int iv = -1;
            for (int w = 0; w < 4; ++w)
                if (V[w][0] == ox && V[w][1] == oy && V[w][2] == oz) iv = w;
            if (iv < 0) continue;
            const uint32_t c = (uint32_t)brick * g.NC + t * B3 + cl;
            const double G00v = G[c], G11v = G[g.C + c], G22v = G[2 * g.C + c], G01v = G[3 * g.C + c],
                         G02v = G[4 * g.C + c], G12v = G[5 * g.C + c];
            double kc[4];
            for (int w = 0; w < 4; ++w) {
                const uint32_t vid = (uint32_t)(cx + V[w][0]) + N1 * ((uint32_t)(cy + V[w][1]) + N1 * (uint32_t)(cz + V[w][2]));
                kc[w] = kv ? kv[vid] : 1.0;
            }
            // the star nodes of this cell: the vertex node iv and the midpoints of its 3 edges
            int sn[4], ss[4];
            sn[0] = iv;
            int ne = 1;
            for (int e = 0; e < 6; ++e)
                if (ea[e] == iv || eb[e] == iv) sn[ne++] = 4 + e;
            for (int a = 0; a < 4; ++a) {
                int X[3] = {0, 0, 0};
                for (int w = 0; w < 4; ++w)
                    for (int d = 0; d < 3; ++d) X[d] += nodes.m[sn[a]][w] * V[w][d];
                ss[a] = star_slot(X[0] - 2 * ox, X[1] - 2 * oy, X[2] - 2 * oz);
            }
            for (int q = 0; q < tab.NQ; ++q) {
                const double kq = tab.lam[q][0] * kc[0] + tab.lam[q][1] * kc[1] + tab.lam[q][2] * kc[2] +
                                  tab.lam[q][3] * kc[3];
                const double wk = tab.w[q] * kq;
                double D[4][3];
                for (int a = 0; a < 4; ++a)
                    for (int d = 0; d < 3; ++d) D[a][d] = tab.D[q][d][sn[a]];
                for (int a = 0; a < 4; ++a) {
                    const double u0 = G00v * D[a][0] + G01v * D[a][1] + G02v * D[a][2];
                    const double u1 = G01v * D[a][0] + G11v * D[a][1] + G12v * D[a][2];
                    const double u2 = G02v * D[a][0] + G12v * D[a][1] + G22v * D[a][2];
                    for (int b = 0; b < 4; ++b)
                        A[ss[a]][ss[b]] += wk * (u0 * D[b][0] + u1 * D[b][1] + u2 * D[b][2]);
                }
            }
        }
    }
    // star dofs outside the lattice or on the boundary: identity rows and columns, zeroed after
    const int Lm = 2 * n;
    bool live[kStar];
    for (int s = 0; s < kStar; ++s) {
        const int c = s == 0 ? 0 : (s <= 7 ? s : s - 7), sg = s <= 7 ? 1 : -1;
        const int X = 2 * vi + sg * (c & 1), Y = 2 * vj + sg * ((c >> 1) & 1), Z = 2 * vk + sg * (c >> 2);
        live[s] = X > 0 && Y > 0 && Z > 0 && X < Lm && Y < Lm && Z < Lm;
    }
    for (int a = 0; a < kStar; ++a)
        for (int b = 0; b < kStar; ++b)
            if (!live[a] || !live[b]) A[a][b] = (a == b) ? 1.0 : 0.0;
    // in-place Gauss-Jordan inverse
    for (int p = 0; p < kStar; ++p) {
        const double piv = 1.0 / A[p][p];
        for (int b = 0; b < kStar; ++b) A[p][b] *= piv;
        A[p][p] = piv;
        for (int a = 0; a < kStar; ++a) {
            if (a == p) continue;
            const double f = A[a][p];
            for (int b = 0; b < kStar; ++b) A[a][b] -= f * A[p][b];
            A[a][p] = -f * piv;
        }
    }
    for (int a = 0; a < kStar; ++a)
        for (int b = 0; b <= a; ++b) {
            const double val = (live[a] && live[b]) ? 0.5 * (A[a][b] + A[b][a]) : 0.0;
            inv[(uint32_t)(a * (a + 1) / 2 + b) * g.NV + v] = (T)val;
        }
}

template <typename T>
__global__ void __launch_bounds__(256) k_patch_local(PatchGeom g, const T* __restrict__ inv, const T* __restrict__ r,
                                                     T* __restrict__ u) {
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= g.NV) return;
    const int n = g.n, N1 = n + 1, Lm = 2 * n;
    const int vi = (int)(v % N1), vj = (int)((v / N1) % N1), vk = (int)(v / (N1 * N1));
    T rs[kStar];
#pragma unroll
    for (int s = 0; s < kStar; ++s) {
        const int c = s == 0 ? 0 : (s <= 7 ? s : s - 7), sg = s <= 7 ? 1 : -1;
        const int X = 2 * vi + sg * (c & 1), Y = 2 * vj + sg * ((c >> 1) & 1), Z = 2 * vk + sg * (c >> 2);
        const bool live = X > 0 && Y > 0 && Z > 0 && X < Lm && Y < Lm && Z < Lm;
        rs[s] = live ? r[(uint32_t)X + g.L * ((uint32_t)Y + g.L * (uint32_t)Z)] : T(0);
    }
    T us[kStar];
#pragma unroll
    for (int a = 0; a < kStar; ++a) us[a] = T(0);
#pragma unroll
    for (int a = 0; a < kStar; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            const T m = inv[(uint32_t)(a * (a + 1) / 2 + b) * g.NV + v];
            us[a] += m * rs[b];
            if (b != a) us[b] += m * rs[a];
        }
#pragma unroll
    for (int a = 0; a < kStar; ++a) u[(uint32_t)a * g.NV + v] = us[a];
}

template <typename T>
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
    const uint32_t dx = X & 1u, dy = Y & 1u, dz = Z & 1u, c = dx + 2 * dy + 4 * dz;
    const uint32_t lo = (X >> 1) + N1 * ((Y >> 1) + N1 * (Z >> 1));
    if (c == 0) {
        z[i] = u[lo];
        return;
    }
    const uint32_t hi = lo + dx + N1 * (dy + N1 * dz);
    z[i] = u[c * g.NV + lo] + u[(7 + c) * g.NV + hi];
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

}  // namespace

size_t patch_bytes(const HostLevel& H, size_t ts) {
    return align256((size_t)kPacked * H.NV * ts) + align256((size_t)kStar * H.NV * ts);
}

template <typename T>
fem_status patch_setup(const fem_mesh& m, int level, const double* k, void* buf, hipStream_t s) {
    const HostLevel& H = m.lev[level];
    const PatchGeom g = patch_geom(H);
    hipLaunchKernelGGL((k_patch_setup<T>), dim3((g.NV + 63) / 64), dim3(64), 0, s, g, dptr<double>(m, H.d_G64), k,
                       reinterpret_cast<T*>(buf));
    return check_launch("fem_patch_setup");
}

template <typename T>
fem_status patch_apply(const fem_mesh& m, int level, void* buf, const T* r, T* z, hipStream_t s) {
    const HostLevel& H = m.lev[level];
    const PatchGeom g = patch_geom(H);
    const T* inv = reinterpret_cast<const T*>(buf);
    T* u = reinterpret_cast<T*>(reinterpret_cast<char*>(buf) + align256((size_t)kPacked * H.NV * sizeof(T)));
    hipLaunchKernelGGL((k_patch_local<T>), dim3((g.NV + 255) / 256), dim3(256), 0, s, g, inv, r, u);
    hipLaunchKernelGGL((k_patch_combine<T>), dim3((unsigned)((H.N + 255) / 256)), dim3(256), 0, s, g,
                       (const T*)u, r, z);
    return check_launch("fem_apply_patch");
}

template fem_status patch_setup<double>(const fem_mesh&, int, const double*, void*, hipStream_t);
template fem_status patch_setup<float>(const fem_mesh&, int, const double*, void*, hipStream_t);
template fem_status patch_apply<double>(const fem_mesh&, int, void*, const double*, double*, hipStream_t);
template fem_status patch_apply<float>(const fem_mesh&, int, void*, const float*, float*, hipStream_t);

}  // namespace fem
