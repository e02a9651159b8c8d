// Cell-wise kernels with a deterministic scatter-add, for gfx950.
//
// Every operator of the method that sums per-cell contributions into shared dofs (the stiffness
// action, its diagonal, the mass action and the adjoint gradient) runs through the same
// two-kernel pattern (the stiffness action on 4-cube bricks replaces step 1 by the cube kernel,
// cube.hpp, for P1/P2 and the lattice kernel, lattice.hpp, for P3):
//
//  1. k_brick: one workgroup per brick of B^3 cubes (6 B^3 cells, one cell per thread).  Each
//     thread gathers its cell's inputs through the structure-of-arrays cell-to-dof map, forms the
//     cell's local output vector (the "producer") and stores it in LDS.  After one barrier each
//     thread sums, for some closure points of the brick, the LDS entries listed for that point in
//     the brick reduction table, in the table's fixed order.  Points strictly inside the brick are
//     owned by it alone and written straight to y; points on the brick's faces are written to a
//     per-brick interface slot.
//  2. k_fixup: one thread per brick-face lattice point sums the interface slots of the 1-8
//     bricks that contain it, in ascending brick order, and writes y.
//
// No atomics and no colour passes: the result is bitwise reproducible for a given mesh, and
// every output entry is written exactly once (so y need not be cleared, and y may alias z in
// the axpby form y = alpha * (A x) + beta * z).
//
// Bricks are dealt to workgroups so that each of the 8 XCDs (separate L2 caches) receives a
// contiguous range of bricks when the brick count is a multiple of 8.
#pragma once
#include <hip/hip_runtime.h>

#include <utility>

#include "common.hpp"
#include "iface.hpp"
#include "incidence.hpp"
#include "tabulate.hpp"

namespace fem {

template <typename T>
struct SArgs {
    int n, nb, Lout;                 // cubes per direction, bricks per direction, output lattice
    int nbx;                         // bricks along x of the interface numbering (nb / R)
    int64_t C;                       // cells of the level the kernel loops over
    const int32_t* map;              // SoA nloc * C (sign bit: boundary dof)
    const T* G;                      // SoA 6 * C
    const T* tab;                    // stiffness tabulation: per point w, lambda[4], D[3][nloc]
    const T* aux;                    // mass: M_ref (nloc^2)
    T* slots;                        // interface partials: 8 arrays (side code) x if_tot points
    uint32_t if_c0, if_c01, if_tot;  // interface points on x planes; + y planes; + z planes
    int mask_cols;                   // gather boundary dofs as zero
    const T* x;                      // input field (u for the gradient)
    const T* x2;                     // second input (lambda for the gradient)
    const T* k;                      // P1 coefficient on the vertex lattice, or null
    T* y;                            // output (may alias z)
    const T* z;
    T alpha, beta;
    int row_mode;                    // RowMode for boundary rows of the output
    const T* xid;                    // values of identity rows
    const double* vxyz;              // cube kernel: vertex coordinates SoA x[nv], y[nv], z[nv]
    uint32_t nv;
    const double* geo;               // cube kernel: the hierarchy's geometry table, or null
    int geo_shift;                   // levels below the coarsest (2^geo_shift cubes per coarsest cube)
    double geo_scale;                // 2^-geo_shift
    int lattice;                     // P3 on 4-cube bricks: dofs addressed by lattice point
};

constexpr int brick_threads(int B) { return B == 4 ? 384 : 64; }

__device__ __forceinline__ int brick_of_block(int bid, int nblocks) {
    if ((nblocks & 7) == 0) {
        const int per = nblocks >> 3;
        return (bid & 7) * per + (bid >> 3);
    }
    return bid;
}

// Integer vertex coordinates of a cell from its brick and local index.
template <int B>
__device__ __forceinline__ void cell_vertices(int bx, int by, int bz, int cl, int V[4][3]) {
    const int cube = cl % (B * B * B), t = cl / (B * B * B);
    V[0][0] = bx * B + cube % B;
    V[0][1] = by * B + (cube / B) % B;
    V[0][2] = bz * B + cube / (B * B);
    const int a0 = (t < 2) ? 0 : (t < 4) ? 1 : 2;
    const int a1 = (t == 0 || t == 5) ? 1 : (t == 1 || t == 3) ? 2 : 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        V[1][k] = V[0][k] + (k == a0);
        V[2][k] = V[1][k] + (k == a1);
        V[3][k] = V[0][k] + 1;
    }
}

// Loads with a 32-bit element offset from a uniform base, so the base stays in scalar registers
// and each lane adds one 32-bit offset (mesh creation keeps every level below 2^29 cells and
// dofs, so each array and each structure-of-arrays plane is addressed within 4 GiB).
template <typename T>
__device__ __forceinline__ T ldg(const T* base, uint32_t idx) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + (uint32_t)(idx * (uint32_t)sizeof(T)));
}
template <typename T>
__device__ __forceinline__ void stg(T* base, uint32_t idx, T v) {
    *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + (uint32_t)(idx * (uint32_t)sizeof(T))) = v;
}
// entry c of plane k of a structure-of-arrays field with C entries per plane
template <typename T>
__device__ __forceinline__ T soa(const T* p, int k, int64_t C, int64_t c) {
    return ldg(p + (size_t)k * (size_t)C, (uint32_t)c);
}

template <typename T>
__device__ __forceinline__ T gather(const T* __restrict__ x, int32_t m, int mask) {
    const uint32_t u = (uint32_t)m;
    const T v = ldg(x, u & 0x7fffffffu);
    return (mask && (m < 0)) ? T(0) : v;
}

// ---------------- producers: the per-cell local vector ----------------

template <int KIND, int P, int B, bool KVAR, typename T>
struct Producer;

// store the brick's partial sum at closure point (la, lb, lc) of brick (bx, by, bz)
template <int PB, typename T>
__device__ __forceinline__ void put_slot(const SArgs<T>& a, int bx, int by, int bz, int la, int lb, int lc, T v) {
    const uint32_t I = (uint32_t)(bx * PB + la), J = (uint32_t)(by * PB + lb), K = (uint32_t)(bz * PB + lc);
    const uint32_t t = iface_index<PB, PB>(I, J, K, (uint32_t)a.Lout, (uint32_t)a.nb, (uint32_t)a.nb, a.if_c0, a.if_c01);
    const uint32_t code = (la == 0 ? 1u : 0u) | (lb == 0 ? 2u : 0u) | (lc == 0 ? 4u : 0u);
    a.slots[(size_t)code * a.if_tot + t] = v;
}

// The cell's stiffness contribution y_K = sum_q w_q k_q D_q^T G D_q x_K from its nodal values,
// G (00, 11, 22, 01, 02, 12) and the coefficient at its vertices (compile-time tabulation, zero
// entries of D generate no instructions).
template <int P, bool KVAR, typename T>
__device__ __forceinline__ void stiffness_local(const T* xs, const T* g, const T* kv, T* out) {
    constexpr int NL = nloc_of(P), NQ = nq_of(P, KVAR);
    constexpr StiffTab<P, KVAR> TB{};
    const T g00 = g[0], g11 = g[1], g22 = g[2], g01 = g[3], g02 = g[4], g12 = g[5];
#pragma unroll
    for (int i = 0; i < NL; ++i) out[i] = T(0);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        T gx = T(0), gy = T(0), gz = T(0);
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            if (TB.D[q][0][i] != 0.0) gx += T(TB.D[q][0][i]) * xs[i];
            if (TB.D[q][1][i] != 0.0) gy += T(TB.D[q][1][i]) * xs[i];
            if (TB.D[q][2][i] != 0.0) gz += T(TB.D[q][2][i]) * xs[i];
        }
        T s = T(TB.w[q]);
        if constexpr (KVAR)
            s *= T(TB.lam[q][0]) * kv[0] + T(TB.lam[q][1]) * kv[1] + T(TB.lam[q][2]) * kv[2] +
                 T(TB.lam[q][3]) * kv[3];
        const T wx = s * (g00 * gx + g01 * gy + g02 * gz);
        const T wy = s * (g01 * gx + g11 * gy + g12 * gz);
        const T wz = s * (g02 * gx + g12 * gy + g22 * gz);
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            T v = out[i];
            if (TB.D[q][0][i] != 0.0) v += T(TB.D[q][0][i]) * wx;
            if (TB.D[q][1][i] != 0.0) v += T(TB.D[q][1][i]) * wy;
            if (TB.D[q][2][i] != 0.0) v += T(TB.D[q][2][i]) * wz;
            out[i] = v;
        }
    }
}

// Stiffness action from the cell-to-dof map and the per-cell factors.
template <int P, int B, bool KVAR, typename T>
struct Producer<K_APPLY, P, B, KVAR, T> {
    static constexpr int NL = nloc_of(P);
    __device__ __forceinline__ static void run(const SArgs<T>& a, int64_t c, int cl, int bx, int by, int bz,
                                               T* out) {
        const int64_t C = a.C;
        T g[6];
#pragma unroll
        for (int e = 0; e < 6; ++e) g[e] = soa(a.G, e, C, c);
        T xs[NL];
#pragma unroll
        for (int i = 0; i < NL; ++i) xs[i] = gather(a.x, soa(a.map, i, C, c), a.mask_cols);
        T kv[4] = {T(1), T(1), T(1), T(1)};
        if constexpr (KVAR) {
            int V[4][3];
            cell_vertices<B>(bx, by, bz, cl, V);
            const int n1 = a.n + 1;
#pragma unroll
            for (int v = 0; v < 4; ++v) kv[v] = a.k[V[v][0] + n1 * (V[v][1] + n1 * V[v][2])];
        }
        stiffness_local<P, KVAR, T>(xs, g, kv, out);
    }
};

// Diagonal: d_i = sum_q w_q k_q (D_q e_i)^T G (D_q e_i).
template <int P, int B, bool KVAR, typename T>
struct Producer<K_DIAG, P, B, KVAR, T> {
    static constexpr int NL = nloc_of(P), NQ = nq_of(P, KVAR), ST = 5 + 3 * NL;
    __device__ __forceinline__ static void run(const SArgs<T>& a, int64_t c, int cl, int bx, int by, int bz,
                                               T* out) {
        const T* __restrict__ tab = a.tab;
        const int64_t C = a.C;
        const T g00 = soa(a.G, 0, C, c), g11 = soa(a.G, 1, C, c), g22 = soa(a.G, 2, C, c);
        const T g01 = soa(a.G, 3, C, c), g02 = soa(a.G, 4, C, c), g12 = soa(a.G, 5, C, c);
        T kv[4] = {T(1), T(1), T(1), T(1)};
        if constexpr (KVAR) {
            int V[4][3];
            cell_vertices<B>(bx, by, bz, cl, V);
            const int n1 = a.n + 1;
#pragma unroll
            for (int v = 0; v < 4; ++v) kv[v] = a.k[V[v][0] + n1 * (V[v][1] + n1 * V[v][2])];
        }
#pragma unroll
        for (int i = 0; i < NL; ++i) out[i] = T(0);
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const T* __restrict__ tq = tab + q * ST;
            T s = tq[0];
            if constexpr (KVAR) s *= tq[1] * kv[0] + tq[2] * kv[1] + tq[3] * kv[2] + tq[4] * kv[3];
#pragma unroll
            for (int i = 0; i < NL; ++i) {
                const T dx = tq[5 + i], dy = tq[5 + NL + i], dz = tq[5 + 2 * NL + i];
                out[i] += s * (g00 * dx * dx + g11 * dy * dy + g22 * dz * dz +
                               T(2) * (g01 * dx * dy + g02 * dx * dz + g12 * dy * dz));
            }
        }
    }
};

// Mass action: y_K = |det J| M_ref x_K, with |det J| = det G.
template <int P, int B, bool KVAR, typename T>
struct Producer<K_MASS, P, B, KVAR, T> {
    static constexpr int NL = nloc_of(P);
    __device__ __forceinline__ static void run(const SArgs<T>& a, int64_t c, int, int, int, int, T* out) {
        const int64_t C = a.C;
        const T g00 = soa(a.G, 0, C, c), g11 = soa(a.G, 1, C, c), g22 = soa(a.G, 2, C, c);
        const T g01 = soa(a.G, 3, C, c), g02 = soa(a.G, 4, C, c), g12 = soa(a.G, 5, C, c);
        const T det = g00 * (g11 * g22 - g12 * g12) - g01 * (g01 * g22 - g12 * g02) + g02 * (g01 * g12 - g11 * g02);
        T xs[NL];
#pragma unroll
        for (int i = 0; i < NL; ++i) xs[i] = gather(a.x, soa(a.map, i, C, c), a.mask_cols);
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            T s = T(0);
#pragma unroll
            for (int j = 0; j < NL; ++j) s += a.aux[i * NL + j] * xs[j];
            out[i] = det * s;
        }
    }
};

// Adjoint gradient, output on the 4 vertices: g_v = - sum_q w_q lambda_v(xi_q)
// (D_q u_K)^T G (D_q l_K).
template <int P, int B, bool KVAR, typename T>
struct Producer<K_GRAD, P, B, KVAR, T> {
    static constexpr int NL = nloc_of(P), NQ = nq_of(P, true), ST = 5 + 3 * NL;
    __device__ __forceinline__ static void run(const SArgs<T>& a, int64_t c, int, int, int, int, T* out) {
        const T* __restrict__ tab = a.tab;
        const int64_t C = a.C;
        const T g00 = soa(a.G, 0, C, c), g11 = soa(a.G, 1, C, c), g22 = soa(a.G, 2, C, c);
        const T g01 = soa(a.G, 3, C, c), g02 = soa(a.G, 4, C, c), g12 = soa(a.G, 5, C, c);
        T us[NL], ls[NL];
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            const int32_t m = soa(a.map, i, C, c);
            us[i] = gather(a.x, m, 1);
            ls[i] = gather(a.x2, m, 1);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) out[v] = T(0);
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const T* __restrict__ tq = tab + q * ST;
            T ux = T(0), uy = T(0), uz = T(0), lx = T(0), ly = T(0), lz = T(0);
#pragma unroll
            for (int i = 0; i < NL; ++i) {
                ux += tq[5 + i] * us[i];
                uy += tq[5 + NL + i] * us[i];
                uz += tq[5 + 2 * NL + i] * us[i];
                lx += tq[5 + i] * ls[i];
                ly += tq[5 + NL + i] * ls[i];
                lz += tq[5 + 2 * NL + i] * ls[i];
            }
            const T s = tq[0] * (ux * (g00 * lx + g01 * ly + g02 * lz) + uy * (g01 * lx + g11 * ly + g12 * lz) +
                                 uz * (g02 * lx + g12 * ly + g22 * lz));
#pragma unroll
            for (int v = 0; v < 4; ++v) out[v] -= tq[1 + v] * s;
        }
    }
};

template <typename T>
__device__ __forceinline__ void finalize(const SArgs<T>& a, uint32_t g, T acc, bool bnd) {
    T v = acc;
    if (bnd) {
        if (a.row_mode == ROW_IDENTITY) v = ldg(a.xid, g);
        else if (a.row_mode == ROW_ZERO) v = T(0);
        else if (a.row_mode == ROW_ONE) v = T(1);
    }
    T r = a.alpha * v;
    if (a.beta != T(0)) r += a.beta * ldg(a.z, g);
    stg(a.y, g, r);
}

// Sum, for every closure point of one type, the LDS entries of the cells that contain it (in the
// fixed order of the incidence table), then write the point: to y if it lies strictly inside the
// brick, else to the brick's interface slot.
template <int PO, int B, int TY, typename T>
__device__ __forceinline__ void reduce_type(const SArgs<T>& a, const T* ys, int brick, int bx, int by, int bz) {
    constexpr Incidence<PO> INC{};
    constexpr int ta = TY % PO, tb = (TY / PO) % PO, tc = TY / (PO * PO);
    constexpr int ea = B + (ta == 0), eb = B + (tb == 0), ec = B + (tc == 0);
    constexpr int NPTS = ea * eb * ec, CNT = INC.cnt[TY];
    constexpr int NC = 6 * B * B * B, NT = brick_threads(B), PB = PO * B;
    const int64_t L = a.Lout;
    for (int idx = threadIdx.x; idx < NPTS; idx += NT) {
        const int ka = idx % ea, kb = (idx / ea) % eb, kc = idx / (ea * eb);
        T acc = T(0);
#pragma unroll
        for (int e = 0; e < CNT; ++e) {
            const int X = ka + INC.dx[TY][e], Y = kb + INC.dy[TY][e], Z = kc + INC.dz[TY][e];
            if (X >= 0 && X < B && Y >= 0 && Y < B && Z >= 0 && Z < B)
                acc += ys[INC.i[TY][e] * NC + INC.t[TY][e] * (B * B * B) + (X + B * (Y + B * Z))];
        }
        const int la = ta + PO * ka, lb = tb + PO * kb, lc = tc + PO * kc;
        if (la == 0 || la == PB || lb == 0 || lb == PB || lc == 0 || lc == PB) {
            put_slot<PB, T>(a, bx, by, bz, la, lb, lc, acc);
        } else {
            const uint32_t g = (uint32_t)(bx * PB + la) + (uint32_t)L * ((uint32_t)(by * PB + lb) + (uint32_t)L * (uint32_t)(bz * PB + lc));
            finalize(a, g, acc, false);
        }
    }
}

template <int PO, int B, typename T, int... TYs>
__device__ __forceinline__ void reduce_all(const SArgs<T>& a, const T* ys, int brick, int bx, int by, int bz,
                                           std::integer_sequence<int, TYs...>) {
    (reduce_type<PO, B, TYs, T>(a, ys, brick, bx, by, bz), ...);
}

template <int KIND, int P, int B, bool KVAR, typename T>
__global__ void __launch_bounds__(brick_threads(B)) k_brick(SArgs<T> a) {
    constexpr int PO = (KIND == K_GRAD) ? 1 : P;
    constexpr int NLO = nloc_of(PO);
    constexpr int NC = 6 * B * B * B;
    constexpr int NT = brick_threads(B);
    __shared__ T ys[NLO * NC];
    const int brick = brick_of_block(blockIdx.x, gridDim.x);
    const int nb = a.nb;
    const int bx = brick % nb, by = (brick / nb) % nb, bz = brick / (nb * nb);
    for (int cl = threadIdx.x; cl < NC; cl += NT) {
        const int64_t c = (int64_t)brick * NC + cl;
        T out[NLO];
        Producer<KIND, P, B, KVAR, T>::run(a, c, cl, bx, by, bz, out);
#pragma unroll
        for (int i = 0; i < NLO; ++i) ys[i * NC + cl] = out[i];
    }
    __syncthreads();
    reduce_all<PO, B, T>(a, ys, brick, bx, by, bz, std::make_integer_sequence<int, PO * PO * PO>{});
}

// Exact unsigned division of n < 2^32 by a runtime divisor d >= 1 via the high half of a 64x64
// product with M = floor((2^64 - 1) / d) + 1 (M = 0 encodes d = 1).
struct Div {
    uint64_t m;
    uint32_t d;
};
inline Div make_div(uint32_t d) { return Div{d == 1 ? 0ull : (~0ull / d) + 1ull, d}; }
__device__ __forceinline__ uint32_t udiv(uint32_t n, Div v) {
    return v.m == 0 ? n : (uint32_t)__umul64hi((uint64_t)n, v.m);
}

struct FixGeom {
    uint32_t cnt0, cnt01, total;   // family boundaries: x planes, + y planes, + z planes
    uint32_t nbx;                  // bricks along x (of span R PB)
    Div L, LL, npx, npxL, npnpx;   // L, L^2, non-x-plane count npx, L npx, np npx
};

// R: bricks merged along x by the kernel that wrote the slots (the x span of a brick is R PB).
template <int PO, int B, int R, typename T>
__global__ void __launch_bounds__(256) k_fixup(SArgs<T> a, FixGeom fg) {
    constexpr int PB = PO * B, PBX = R * PB;
    const uint32_t t = blockIdx.x * 256u + threadIdx.x;
    if (t >= fg.total) return;
    const uint32_t L = fg.L.d, nb = (uint32_t)a.nb, nbx = fg.nbx, npx = fg.npx.d;
    uint32_t I, J, K;
    if (t < fg.cnt0) {
        const uint32_t pl = udiv(t, fg.LL), r = t - pl * fg.LL.d;
        I = pl * PBX;
        K = udiv(r, fg.L);
        J = r - K * L;
    } else if (t < fg.cnt01) {
        const uint32_t u = t - fg.cnt0;
        const uint32_t pl = udiv(u, fg.npxL), r = u - pl * fg.npxL.d;
        J = pl * PB;
        K = udiv(r, fg.npx);
        const uint32_t iu = r - K * npx;
        if constexpr (PBX > 1) I = (iu / (PBX - 1)) * PBX + iu % (PBX - 1) + 1; else I = iu;
    } else {
        const uint32_t u = t - fg.cnt01;
        const uint32_t pl = udiv(u, fg.npnpx), r = u - pl * fg.npnpx.d;
        K = pl * PB;
        const uint32_t ju = udiv(r, fg.npx), iu = r - ju * npx;
        if constexpr (PBX > 1) I = (iu / (PBX - 1)) * PBX + iu % (PBX - 1) + 1; else I = iu;
        if constexpr (PB > 1) J = (ju / (PB - 1)) * PB + ju % (PB - 1) + 1; else J = ju;
    }
    const uint32_t g = I + L * (J + L * K);
    const bool bnd = I == 0 || J == 0 || K == 0 || I == L - 1 || J == L - 1 || K == L - 1;
    // a boundary row whose value the row mode replaces needs no slots; its identity value and z
    // are read before the sum, so every load of the thread is in flight at once
    const bool need = !(bnd && a.row_mode != ROW_NONE);
    const T xv = (bnd && a.row_mode == ROW_IDENTITY) ? ldg(a.xid, g) : T(0);
    const T zv = (a.beta != T(0)) ? ldg(a.z, g) : T(0);
    // Along each axis the point has a lower-brick candidate (side bit 0: valid off a brick plane,
    // or on a plane above the first brick) and an upper-brick candidate (side bit 1: on a plane
    // below the last brick).  The bricks containing the point, in ascending brick order (z, then
    // y, then x), are therefore the side codes 0..7 whose three bits are valid: all eight
    // (predicated) loads are issued together and summed in code order.
    const uint32_t X[3] = {I, J, K};
    bool lo[3], hi[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const uint32_t span = d == 0 ? PBX : PB, nbd = d == 0 ? nbx : nb;
        const uint32_t q = X[d] / span, r = X[d] - q * span;
        lo[d] = r != 0 || q >= 1;
        hi[d] = r == 0 && q < nbd;
    }
    T v[8];
#pragma unroll
    for (int code = 0; code < 8; ++code) {
        const bool ok = need && ((code & 1) ? hi[0] : lo[0]) && ((code & 2) ? hi[1] : lo[1]) &&
                        ((code & 4) ? hi[2] : lo[2]);
        v[code] = ok ? a.slots[(size_t)code * fg.total + t] : T(0);
    }
    T acc = v[0];
#pragma unroll
    for (int code = 1; code < 8; ++code) acc += v[code];
    if (bnd) {
        if (a.row_mode == ROW_IDENTITY) acc = xv;
        else if (a.row_mode == ROW_ZERO) acc = T(0);
        else if (a.row_mode == ROW_ONE) acc = T(1);
    }
    T r = a.alpha * acc;
    if (a.beta != T(0)) r += a.beta * zv;
    stg(a.y, g, r);
}

}  // namespace fem
