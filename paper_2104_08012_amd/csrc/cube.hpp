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

// The six tetrahedra of a cube split into two halves {0,1,2} and {3,4,5}; wave h of the workgroup
// computes half h of every cube of the brick, so each thread keeps only the lattice points its three
// cells touch.
template <int P>
struct HalfPoints {
    static constexpr int NCP = (P + 1) * (P + 1) * (P + 1);
    bool touched[2][NCP];
    constexpr HalfPoints() : touched{} {
        const CubeNodes<P> cn{};
        for (int t = 0; t < 6; ++t)
            for (int i = 0; i < nloc_of(P); ++i) touched[t / 3][cn.cp[t][i]] = true;
    }
};

template <int H, int P, int B, bool KVAR, typename T>
__device__ __forceinline__ void cube_half(const SArgs<T>& a, const T* sx, T* acc, uint32_t c0, int base, int par,
                                          const T* kc) {
    constexpr int NL = nloc_of(P), NQ = nq_of(P, KVAR), PC = P + 1, NCP = PC * PC * PC, NT = B * B * B;
    constexpr int QS = P * B + 1;
    constexpr StiffTab<P, KVAR> TB{};
    constexpr CubeNodes<P> CN{};
    constexpr HalfPoints<P> HP{};
    const uint32_t C = (uint32_t)a.C;
    T ys[NCP];
#pragma unroll
    for (int j = 0; j < NCP; ++j) ys[j] = T(0);
#pragma unroll
    for (int t = 3 * H; t < 3 * H + 3; ++t) {
        const uint32_t c = c0 + (uint32_t)(t * NT);
        const T g00 = ldg(a.G, c), g11 = ldg(a.G, C + c), g22 = ldg(a.G, 2 * C + c);
        const T g01 = ldg(a.G, 3 * C + c), g02 = ldg(a.G, 4 * C + c), g12 = ldg(a.G, 5 * C + c);
        T xt[NL];
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            const int j = CN.cp[t][i];
            xt[i] = sx[base + (j % PC) + QS * (((j / PC) % PC) + QS * (j / (PC * PC)))];
        }
        T kt[4];
        if constexpr (KVAR) {
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
                if (TB.D[q][0][i] != 0.0) gx += T(TB.D[q][0][i]) * xt[i];
                if (TB.D[q][1][i] != 0.0) gy += T(TB.D[q][1][i]) * xt[i];
                if (TB.D[q][2][i] != 0.0) gz += T(TB.D[q][2][i]) * xt[i];
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
                T v = ys[CN.cp[t][i]];
                if (TB.D[q][0][i] != 0.0) v += T(TB.D[q][0][i]) * wx;
                if (TB.D[q][1][i] != 0.0) v += T(TB.D[q][1][i]) * wy;
                if (TB.D[q][2][i] != 0.0) v += T(TB.D[q][2][i]) * wz;
                ys[CN.cp[t][i]] = v;
            }
        }
    }
    // cubes of one parity share no lattice point; this wave adds its cubes parity by parity.  The
    // wave's LDS operations complete in issue order, and the empty asm with a memory clobber keeps
    // the compiler from moving a later phase's reads above an earlier phase's writes.
#pragma unroll
    for (int ph = 0; ph < 8; ++ph) {
        if (par == ph) {
#pragma unroll
            for (int j = 0; j < NCP; ++j) {
                if (!HP.touched[H][j]) continue;
                const int off = (j % PC) + QS * (((j / PC) % PC) + QS * (j / (PC * PC)));
                acc[base + off] += ys[j];
            }
        }
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    }
}

#ifndef FEM_CUBE_MIN_WAVES
#define FEM_CUBE_MIN_WAVES 1
#endif
template <int P, int B, bool KVAR, typename T>
__global__ void __launch_bounds__(2 * B * B * B, (KVAR ? 1 : FEM_CUBE_MIN_WAVES)) k_cube_apply(SArgs<T> a) {
    static_assert(B * B * B == 64, "one wave per half-brick");
    constexpr int NT = B * B * B, NTH = 2 * NT, PB = P * B, QS = PB + 1, Q = QS * QS * QS, QB = box_slots<PB>();
    __shared__ T sx[Q];
    __shared__ T acc0[Q];
    __shared__ T acc1[Q];
    const int brick = brick_of_block(blockIdx.x, gridDim.x);
    const int nb = a.nb;
    const int bx = brick % nb, by = (brick / nb) % nb, bz = brick / (nb * nb);
    const int half = threadIdx.x / NT;            // wave-uniform
    const int cube = threadIdx.x % NT;
    const int lx = cube % B, ly = (cube / B) % B, lz = cube / (B * B);
    const uint32_t C = (uint32_t)a.C;
    const uint32_t cb = (uint32_t)brick * 6u * NT;
    // the brick's closure dofs, each gathered once through the map of the first cell reaching it
    for (int q = threadIdx.x; q < Q; q += NTH) {
        acc0[q] = T(0);
        acc1[q] = T(0);
        const int32_t f = ldg(a.gfirst, (uint32_t)q);
        const int32_t m = ldg(a.map, (uint32_t)(f >> 16) * C + cb + (uint32_t)(f & 0xffff));
        const T v = ldg(a.x, (uint32_t)m & 0x7fffffffu);
        sx[q] = (a.mask_cols && m < 0) ? T(0) : v;
    }
    T kc[8];
    if constexpr (KVAR) {
        const int n1 = a.n + 1;
        const int vx = bx * B + lx, vy = by * B + ly, vz = bz * B + lz;
#pragma unroll
        for (int j = 0; j < 8; ++j)
            kc[j] = ldg(a.k, (uint32_t)((vx + (j & 1)) + n1 * ((vy + ((j >> 1) & 1)) + n1 * (vz + (j >> 2)))));
    }
    __syncthreads();
    const int par = (lx & 1) | ((ly & 1) << 1) | ((lz & 1) << 2);
    const int base = (P * lx) + QS * ((P * ly) + QS * (P * lz));
    const uint32_t c0 = cb + (uint32_t)cube;
    if (half == 0) cube_half<0, P, B, KVAR, T>(a, sx, acc0, c0, base, par, kc);
    else cube_half<1, P, B, KVAR, T>(a, sx, acc1, c0, base, par, kc);
    __syncthreads();
    // write the closure row by row (rows along x): interior points of interior rows go to y as
    // a contiguous run, every other point to its interface slot
    const int64_t L = a.Lout;
    constexpr int QI = QS - 2;
    for (int r = threadIdx.x; r < QS * QS; r += NTH) {
        const int lb = r % QS, lc = r / QS;
        T row[QS];
#pragma unroll
        for (int la = 0; la < QS; ++la) row[la] = acc0[QS * r + la] + acc1[QS * r + la];
        T* sl = a.slots + (size_t)brick * QB;
        if (lc == 0 || lc == PB) {
            const int s0 = (lc == 0 ? 0 : QS * QS) + QS * lb;
#pragma unroll
            for (int la = 0; la < QS; ++la) sl[s0 + la] = row[la];
        } else if (lb == 0 || lb == PB) {
            const int s0 = 2 * QS * QS + (lb == 0 ? 0 : QS * QI) + QS * (lc - 1);
#pragma unroll
            for (int la = 0; la < QS; ++la) sl[s0 + la] = row[la];
        } else {
            const int s0 = 2 * QS * QS + 2 * QS * QI + (lb - 1) + QI * (lc - 1);
            sl[s0] = row[0];
            sl[s0 + QI * QI] = row[PB];
            const int64_t g0 = (bx * PB) + L * ((by * PB + lb) + L * (int64_t)(bz * PB + lc));
#pragma unroll
            for (int la = 1; la < PB; ++la) finalize(a, g0 + la, row[la], false);
        }
    }
}

}  // namespace fem
