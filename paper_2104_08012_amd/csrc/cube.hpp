// Stiffness action for P1 and P2 with one thread per cube (the cube's six tetrahedra).
//
// Same result and the same deterministic two-kernel scheme as k_brick (brick workgroups, interior
// points written directly, brick-face points through interface slots and k_fixup), organised to
// cut instructions on gfx950's 64-wide VALU:
//  * a thread gathers the cube's (p+1)^3 distinct dofs once (8 for P1, 27 for P2) instead of 6 nloc
//    per-cell gathers, through the structure-of-arrays cell-to-dof map of the first cell that
//    reaches each point;
//  * the six cells' contributions accumulate in registers at the cube's lattice points (the
//    node-to-point map is a compile-time table);
//  * quadrature tabulations are literals, so zero gradient entries generate no instructions;
//  * cubes are summed into the brick's closure in LDS in 8 phases by cube parity (cubes of one
//    parity share no point), a fixed order, so the result is reproducible;
//  * loads use 32-bit offsets from uniform bases.
#pragma once
#include "scatter.hpp"
#include "tabulate.hpp"

namespace fem {

// load with a 32-bit byte offset from a uniform base (scalar-base addressing)
template <typename T>
__device__ __forceinline__ T ldg(const T* base, uint32_t idx) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + (uint32_t)(idx * (uint32_t)sizeof(T)));
}

#ifndef FEM_CUBE_MIN_WAVES
#define FEM_CUBE_MIN_WAVES 1
#endif
template <int P, int B, bool KVAR, typename T>
__global__ void __launch_bounds__(B * B * B, FEM_CUBE_MIN_WAVES) k_cube_apply(SArgs<T> a) {
    constexpr int NL = nloc_of(P), NQ = nq_of(P, KVAR), PC = P + 1, NCP = PC * PC * PC;
    constexpr int NT = B * B * B, PB = P * B, QS = PB + 1, Q = QS * QS * QS;
    constexpr StiffTab<P, KVAR> TB{};
    constexpr CubeNodes<P> CN{};
    __shared__ T acc[Q];
    const int brick = brick_of_block(blockIdx.x, gridDim.x);
    const int nb = a.nb;
    const int bx = brick % nb, by = (brick / nb) % nb, bz = brick / (nb * nb);
    const int cube = threadIdx.x;
    const int lx = cube % B, ly = (cube / B) % B, lz = cube / (B * B);
    for (int q = threadIdx.x; q < Q; q += NT) acc[q] = T(0);

    const uint32_t C = (uint32_t)a.C;
    const uint32_t c0 = (uint32_t)(brick * 6 * NT + cube);    // cell of tetrahedron t: c0 + t * NT
    // gather the cube's distinct dofs
    T xs[NCP];
#pragma unroll
    for (int j = 0; j < NCP; ++j) {
        const int32_t m = ldg(a.map, (uint32_t)CN.first_i[j] * C + c0 + (uint32_t)(CN.first_t[j] * NT));
        const T v = ldg(a.x, (uint32_t)m & 0x7fffffffu);
        xs[j] = (a.mask_cols && m < 0) ? T(0) : v;
    }
    T kc[8];
    if constexpr (KVAR) {
        const int n1 = a.n + 1;
        const int vx = bx * B + lx, vy = by * B + ly, vz = bz * B + lz;
#pragma unroll
        for (int j = 0; j < 8; ++j)
            kc[j] = ldg(a.k, (uint32_t)((vx + (j & 1)) + n1 * ((vy + ((j >> 1) & 1)) + n1 * (vz + (j >> 2)))));
    }
    T ys[NCP];
#pragma unroll
    for (int j = 0; j < NCP; ++j) ys[j] = T(0);
#pragma unroll
    for (int t = 0; t < 6; ++t) {
        const uint32_t c = c0 + (uint32_t)(t * NT);
        const T g00 = ldg(a.G, c), g11 = ldg(a.G, C + c), g22 = ldg(a.G, 2 * C + c);
        const T g01 = ldg(a.G, 3 * C + c), g02 = ldg(a.G, 4 * C + c), g12 = ldg(a.G, 5 * C + c);
        T kt[4];
        if constexpr (KVAR) {
            // vertex v of the path tetrahedron at cube corner: v0 = 0, v1 = e_s0, v2 = e_s0 + e_s1, v3 = 7
            const int s0 = perm_axis(t, 0), s1 = perm_axis(t, 1);
            kt[0] = kc[0];
            kt[1] = kc[1 << s0];
            kt[2] = kc[(1 << s0) | (1 << s1)];
            kt[3] = kc[7];
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            T gx = T(0), gy = T(0), gz = T(0);
#pragma unroll
            for (int i = 0; i < NL; ++i) {
                const T xv = xs[CN.cp[t][i]];
                if (TB.D[q][0][i] != 0.0) gx += T(TB.D[q][0][i]) * xv;
                if (TB.D[q][1][i] != 0.0) gy += T(TB.D[q][1][i]) * xv;
                if (TB.D[q][2][i] != 0.0) gz += T(TB.D[q][2][i]) * xv;
            }
            T s = T(TB.w[q]);
            if constexpr (KVAR)
                s *= T(TB.lam[q][0]) * kt[0] + T(TB.lam[q][1]) * kt[1] + T(TB.lam[q][2]) * kt[2] +
                     T(TB.lam[q][3]) * kt[3];
            const T wx = s * (g00 * gx + g01 * gy + g02 * gz);
            const T wy = s * (g01 * gx + g11 * gy + g12 * gz);
            const T wz = s * (g02 * gx + g12 * gy + g22 * gz);
#pragma unroll
            for (int i = 0; i < NL; ++i) {
                T acc_i = ys[CN.cp[t][i]];
                if (TB.D[q][0][i] != 0.0) acc_i += T(TB.D[q][0][i]) * wx;
                if (TB.D[q][1][i] != 0.0) acc_i += T(TB.D[q][1][i]) * wy;
                if (TB.D[q][2][i] != 0.0) acc_i += T(TB.D[q][2][i]) * wz;
                ys[CN.cp[t][i]] = acc_i;
            }
        }
    }
    __syncthreads();
    // cubes of equal parity share no lattice point: add them into the closure phase by phase
    const int par = (lx & 1) | ((ly & 1) << 1) | ((lz & 1) << 2);
    const int base = (P * lx) + QS * ((P * ly) + QS * (P * lz));
#pragma unroll
    for (int ph = 0; ph < 8; ++ph) {
        if (par == ph) {
#pragma unroll
            for (int j = 0; j < NCP; ++j) {
                const int off = (j % PC) + QS * (((j / PC) % PC) + QS * (j / (PC * PC)));
                acc[base + off] += ys[j];
            }
        }
        __syncthreads();
    }
    // write the closure row by row (rows along x): interior points of interior rows go to y as
    // a contiguous run, brick-face points to their interface slots
    const int64_t L = a.Lout;
    for (int r = threadIdx.x; r < QS * QS; r += NT) {
        const int lb = r % QS, lc = r / QS;
        const T* row = &acc[QS * r];
        if (lc == 0 || lc == PB || lb == 0 || lb == PB) {
#pragma unroll
            for (int la = 0; la < QS; ++la) put_slot<PB, T>(a, bx, by, bz, la, lb, lc, row[la]);
        } else {
            put_slot<PB, T>(a, bx, by, bz, 0, lb, lc, row[0]);
            put_slot<PB, T>(a, bx, by, bz, PB, lb, lc, row[PB]);
            const int64_t g0 = (bx * PB) + L * ((by * PB + lb) + L * (int64_t)(bz * PB + lc));
#pragma unroll
            for (int la = 1; la < PB; ++la) finalize(a, g0 + la, row[la], false);
        }
    }
}

}  // namespace fem
