// Stiffness action for P3 on 4-cube bricks with the dofs addressed by lattice point.
//
// One workgroup per brick and one thread per tetrahedron, as k_brick, with the same brick
// reduction and interface slots (so the same k_fixup finishes the brick faces), but without
// the per-cell tables the general kernel reads:
//  * the dofs of a level are numbered by their lattice point, g = I + L (J + L K), so the
//    workgroup stages the brick's closure of (4p + 1)^3 values of x in LDS with coalesced loads
//    (boundary values as zero when columns are masked), and node i of a tetrahedron with
//    vertices V_0 + D_w is the closure point p (cube corner) + m_i1 D_1 + m_i2 D_2 + m_i3 D_3
//    (m_i the node's multi-index, D_1 = e_s0, D_2 = e_s0 + e_s1, D_3 = (1, 1, 1)): the
//    tetrahedron type is the wave's (64 cubes per type), so each read is the lane's cube offset
//    plus a wave-uniform one;
//  * on refined levels whose bricks lie in one coarsest cube (GEO) the geometric factors come from
//    the coarsest level's table (staged in LDS, scaled by 2^-level), found by ordering the
//    tetrahedron's centroid inside the coarsest cube; otherwise from the per-cell factors;
//  * a P1 coefficient is staged at the brick's 5^3 vertices.
// The closure values and the cells' results share one LDS array (the results are written once
// every thread has read its nodal values).
#pragma once
#include "scatter.hpp"

namespace fem {

template <int P, bool KVAR, bool GEO, typename T>
__global__ void __launch_bounds__(384) k_lattice_apply(SArgs<T> a) {
    constexpr int B = 4, NL = nloc_of(P), NC = 6 * B * B * B, NT = brick_threads(B), PB = P * B;
    constexpr int QS = PB + 1, PS = QS * QS, NQ3 = QS * PS;   // closure: la + QS lb + PS lc
    constexpr int VS = B + 1, NV3 = VS * VS * VS, NG = 216;
    static_assert(NT == NC, "one thread per tetrahedron of the brick");
    static_assert(NQ3 <= NL * NC, "the closure fits in the results array");
    constexpr NodeList<P> ND{};
    __shared__ T ys[NL * NC];
    __shared__ T gt[GEO ? NG : 1];
    __shared__ T kl[KVAR ? NV3 : 1];
    const int brick = brick_of_block(blockIdx.x, gridDim.x);
    const int nb = a.nb;
    const int bx = brick % nb, by = (brick / nb) % nb, bz = brick / (nb * nb);
    const int tid = threadIdx.x;
    const uint32_t Lo = (uint32_t)a.Lout;

    // ---- stage the closure of x, the geometry table and the vertex coefficient ----
    {
        constexpr int NIT = (NQ3 + NT - 1) / NT;
        const uint32_t I0 = (uint32_t)(bx * PB), J0 = (uint32_t)(by * PB), K0 = (uint32_t)(bz * PB);
        T v[NIT];
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int r = (tid + NT * it < NQ3) ? tid + NT * it : NQ3 - 1;
            const uint32_t I = I0 + (uint32_t)(r % QS), J = J0 + (uint32_t)((r / QS) % QS), K = K0 + (uint32_t)(r / PS);
            v[it] = ldg(a.x, I + Lo * (J + Lo * K));
            if (a.mask_cols && (I == 0 || J == 0 || K == 0 || I == Lo - 1 || J == Lo - 1 || K == Lo - 1)) v[it] = T(0);
        }
        double gv = 0.0;
        if constexpr (GEO) {
            const int sh = a.geo_shift;
            const uint32_t n0 = (uint32_t)a.n >> sh;
            const uint32_t q0 = (uint32_t)((bx * B) >> sh) + n0 * ((uint32_t)((by * B) >> sh) + n0 * (uint32_t)((bz * B) >> sh));
            gv = ldg(a.geo, q0 * (uint32_t)NG + (uint32_t)(tid < NG ? tid : NG - 1));
        }
        T kv = T(0);
        if constexpr (KVAR) {
            const int r = tid < NV3 ? tid : NV3 - 1;
            const uint32_t n1 = (uint32_t)a.n + 1;
            const uint32_t w = (uint32_t)(bx * B + r % VS) + n1 * ((uint32_t)(by * B + (r / VS) % VS) + n1 * (uint32_t)(bz * B + r / (VS * VS)));
            kv = ldg(a.k, w);
        }
#pragma unroll
        for (int it = 0; it < NIT; ++it)
            if (tid + NT * it < NQ3) ys[tid + NT * it] = v[it];
        if constexpr (GEO)
            if (tid < NG) gt[tid] = T(gv * a.geo_scale);
        if constexpr (KVAR)
            if (tid < NV3) kl[tid] = kv;
    }
    __syncthreads();

    // ---- the thread's tetrahedron: type t (the wave's), cube (lx, ly, lz) ----
    const int t = __builtin_amdgcn_readfirstlane(tid / (B * B * B));
    const int cube = tid % (B * B * B);
    const int lx = cube % B, ly = (cube / B) % B, lz = cube / (B * B);
    const int s0 = perm_axis(t, 0), s1 = perm_axis(t, 1);
    const int c0 = s0 == 0 ? 1 : s0 == 1 ? QS : PS, c1 = s1 == 0 ? 1 : s1 == 1 ? QS : PS;   // closure strides
    const int xb = P * (lx + QS * ly + PS * lz);
    T xs[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i) {
        const int m1 = ND.m[i][1], m2 = ND.m[i][2], m3 = ND.m[i][3];
        xs[i] = ys[xb + m3 * (1 + QS + PS) + (m1 + m2) * c0 + m2 * c1];
    }
    T g[6];
    if constexpr (GEO) {
        const int msk = (1 << a.geo_shift) - 1;
        const int u[3] = {4 * ((bx * B + lx) & msk), 4 * ((by * B + ly) & msk), 4 * ((bz * B + lz) & msk)};
        const int ux = u[0] + centroid4(t, 0), uy = u[1] + centroid4(t, 1), uz = u[2] + centroid4(t, 2);
        const int t0 = (kPathTypeCode >> (3 * ((ux > uy) + 2 * (ux > uz) + 4 * (uy > uz)))) & 7;
#pragma unroll
        for (int e = 0; e < 6; ++e) g[e] = gt[6 * (6 * t0 + t) + e];
    } else {
        const int64_t c = (int64_t)brick * NC + tid;
#pragma unroll
        for (int e = 0; e < 6; ++e) g[e] = soa(a.G, e, a.C, c);
    }
    T kv[4] = {T(1), T(1), T(1), T(1)};
    if constexpr (KVAR) {
        const int v0 = lx + VS * (ly + VS * lz);
        const int k0 = s0 == 0 ? 1 : s0 == 1 ? VS : VS * VS, k1 = s1 == 0 ? 1 : s1 == 1 ? VS : VS * VS;
        kv[0] = kl[v0];
        kv[1] = kl[v0 + k0];
        kv[2] = kl[v0 + k0 + k1];
        kv[3] = kl[v0 + 1 + VS + VS * VS];
    }
    T out[NL];
    stiffness_local<P, KVAR, T>(xs, g, kv, out);
    __syncthreads();   // every thread has read its nodal values: the results overwrite the closure
#pragma unroll
    for (int i = 0; i < NL; ++i) ys[i * NC + tid] = out[i];
    __syncthreads();
    reduce_all<P, B, T>(a, ys, brick, bx, by, bz, std::make_integer_sequence<int, P * P * P>{});
}

}  // namespace fem
