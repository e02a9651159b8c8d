// Stiffness action for P1 and P2 with one thread per cube (the cube's six tetrahedra).
//
// Same result and the same deterministic two-kernel scheme as k_brick (brick workgroups, interior
// points written directly, brick-face points through interface slots and k_fixup), organised to
// cut memory traffic and instructions on gfx950's 64-wide VALU:
//  * a thread gathers the cube's (p+1)^3 distinct dofs once (8 for P1, 27 for P2) through a per-cube
//    structure-of-arrays dof map (entry j of every cube contiguous), instead of 6 nloc per-cell
//    gathers;
//  * the geometry is computed in the kernel from the FP64 coordinates of the cube's 8 vertices:
//    for each tetrahedron the edge vectors e1, e2, e3 from its first vertex, the cofactor rows
//    c1 = e2 x e3, c2 = e3 x e1, c3 = e1 x e2 (so that J^-1 has rows c_a / det), det = e1 . c1,
//    and G = |det| J^-1 J^-T = [c_a . c_b] / |det|.  No per-cell geometric factors are read;
//  * the six cells' contributions accumulate in registers at the cube's lattice points (the
//    node-to-point map is a compile-time table);
//  * quadrature tabulations are literals, so zero gradient entries generate no instructions;
//  * the cubes' point values go to LDS once; then each closure point of the brick sums the values
//    of the (up to 8) cubes containing it in a fixed order (so the result is reproducible), one
//    lane per row of points along x with the x loop unrolled; the sums return to LDS and are
//    written with consecutive lanes on consecutive points, so stores to y are contiguous runs;
//  * loads use 32-bit offsets from uniform bases (the host keeps such levels below 4 GiB per array).
#pragma once
#include "scatter.hpp"
#include "tabulate.hpp"

namespace fem {

// load with a 32-bit byte offset from a uniform base (scalar-base addressing)
template <typename T>
__device__ __forceinline__ T ldg(const T* base, uint32_t idx) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + (uint32_t)(idx * (uint32_t)sizeof(T)));
}

// Contributions along one axis to closure coordinate l of a brick (lattice spacing h/P, cubes
// 0..B-1): the cube with l / P and local index l % P, and, where l is a cube boundary above the
// first, also the cube below with local index P.  off = local index * sj * B^3 + cube * sc is the
// axis's share of the LDS offset (sj, sc: strides of the local point and cube indices).
template <int P, int B>
__device__ __forceinline__ void axis_terms(int l, int sj, int sc, int off[2], bool valid[2]) {
    constexpr int NT = B * B * B;
    const int c0 = l / P, a0 = l % P;
    valid[0] = c0 < B;
    off[0] = a0 * sj * NT + c0 * sc;
    valid[1] = a0 == 0 && c0 > 0;
    off[1] = P * sj * NT + (c0 - 1) * sc;
}

// 1 / d from the hardware reciprocal refined by two Newton steps r <- r + r (1 - d r) (quadratic
// convergence: well below an ulp of error left for the accuracy the kernels need).
__device__ __forceinline__ double recip(double d) {
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    e = fma(-d, r, 1.0);
    return fma(r, e, r);
}

#ifndef FEM_CUBE_MIN_WAVES
#define FEM_CUBE_MIN_WAVES 2
#endif
template <int P, int B, bool KVAR, typename T>
__global__ void __launch_bounds__(B * B * B, FEM_CUBE_MIN_WAVES) k_cube_apply(SArgs<T> a) {
    constexpr int NL = nloc_of(P), NQ = nq_of(P, KVAR), PC = P + 1, NCP = PC * PC * PC;
    constexpr int NT = B * B * B, PB = P * B, QS = PB + 1;
    constexpr StiffTab<P, KVAR> TB{};
    constexpr CubeNodes<P> CN{};
    constexpr int ZERO = NCP * NT;
    __shared__ T part[NCP * NT + 1];   // cube point j of cube c at part[j * NT + c]; last: zero
    const int brick = brick_of_block(blockIdx.x, gridDim.x);
    const int nb = a.nb;
    const int bx = brick % nb, by = (brick / nb) % nb, bz = brick / (nb * nb);
    const int cube = threadIdx.x;
    const int lx = cube % B, ly = (cube / B) % B, lz = cube / (B * B);

    const uint32_t NCB = a.ncube;
    const uint32_t cid = (uint32_t)(brick * NT + cube);
    // gather the cube's distinct dofs
    T xs[NCP];
#pragma unroll
    for (int j = 0; j < NCP; ++j) {
        const int32_t m = ldg(a.cmap, (uint32_t)j * NCB + cid);
        const T v = ldg(a.x, (uint32_t)m & 0x7fffffffu);
        xs[j] = (a.mask_cols && m < 0) ? T(0) : v;
    }
    // corner coordinates relative to corner 0 (corner j at offset (j & 1, j >> 1 & 1, j >> 2))
    const uint32_t n1 = (uint32_t)a.n + 1, NV = a.nv;
    const uint32_t v0 = (uint32_t)(bx * B + lx) + n1 * ((uint32_t)(by * B + ly) + n1 * (uint32_t)(bz * B + lz));
    double D[8][3];
    {
        const double p0x = ldg(a.vxyz, v0), p0y = ldg(a.vxyz, NV + v0), p0z = ldg(a.vxyz, 2 * NV + v0);
#pragma unroll
        for (int j = 1; j < 8; ++j) {
            const uint32_t v = v0 + (uint32_t)(j & 1) + n1 * ((uint32_t)((j >> 1) & 1) + n1 * (uint32_t)(j >> 2));
            D[j][0] = ldg(a.vxyz, v) - p0x;
            D[j][1] = ldg(a.vxyz, NV + v) - p0y;
            D[j][2] = ldg(a.vxyz, 2 * NV + v) - p0z;
        }
    }
    T kc[8];
    if constexpr (KVAR) {
#pragma unroll
        for (int j = 0; j < 8; ++j)
            kc[j] = ldg(a.k, v0 + (uint32_t)(j & 1) + n1 * ((uint32_t)((j >> 1) & 1) + n1 * (uint32_t)(j >> 2)));
    }
    T ys[NCP];
#pragma unroll
    for (int j = 0; j < NCP; ++j) ys[j] = T(0);
#pragma unroll
    for (int t = 0; t < 6; ++t) {
        // path tetrahedron: v0 = corner 0, v1 = e_s0, v2 = e_s0 + e_s1, v3 = corner 7
        const int s0 = perm_axis(t, 0), s1 = perm_axis(t, 1);
        const int j1 = 1 << s0, j2 = (1 << s0) | (1 << s1);
        const double* e1 = D[j1];
        const double* e2 = D[j2];
        const double* e3 = D[7];
        const double c1x = e2[1] * e3[2] - e2[2] * e3[1], c1y = e2[2] * e3[0] - e2[0] * e3[2],
                     c1z = e2[0] * e3[1] - e2[1] * e3[0];
        const double c2x = e3[1] * e1[2] - e3[2] * e1[1], c2y = e3[2] * e1[0] - e3[0] * e1[2],
                     c2z = e3[0] * e1[1] - e3[1] * e1[0];
        const double c3x = e1[1] * e2[2] - e1[2] * e2[1], c3y = e1[2] * e2[0] - e1[0] * e2[2],
                     c3z = e1[0] * e2[1] - e1[1] * e2[0];
        const double det = e1[0] * c1x + e1[1] * c1y + e1[2] * c1z;
        constexpr double kScale = (P == 2 && !KVAR) ? 1.0 / 120.0 : 1.0;   // P1 mass factor, vertex form
        const double inv = kScale * recip(fabs(det));
        const T g00 = T((c1x * c1x + c1y * c1y + c1z * c1z) * inv);
        const T g11 = T((c2x * c2x + c2y * c2y + c2z * c2z) * inv);
        const T g22 = T((c3x * c3x + c3y * c3y + c3z * c3z) * inv);
        const T g01 = T((c1x * c2x + c1y * c2y + c1z * c2z) * inv);
        const T g02 = T((c1x * c3x + c1y * c3y + c1z * c3z) * inv);
        const T g12 = T((c2x * c3x + c2y * c3y + c2z * c3z) * inv);
        T kt[4];
        if constexpr (KVAR) {
            kt[0] = kc[0];
            kt[1] = kc[j1];
            kt[2] = kc[j2];
            kt[3] = kc[7];
        }
        if constexpr (P == 2 && !KVAR) {
            // reference gradient at the vertices, w_v = G g_v, mixed by the P1 mass matrix
            // (the factor 1/120 is in G), then the transposed product
            constexpr VertexGrad<P> VG{};
            T hx[4], hy[4], hz[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                T gx = T(0), gy = T(0), gz = T(0);
#pragma unroll
                for (int i = 0; i < NL; ++i) {
                    const T xv = xs[CN.cp[t][i]];
                    if (VG.D[v][0][i] != 0.0) gx += T(VG.D[v][0][i]) * xv;
                    if (VG.D[v][1][i] != 0.0) gy += T(VG.D[v][1][i]) * xv;
                    if (VG.D[v][2][i] != 0.0) gz += T(VG.D[v][2][i]) * xv;
                }
                hx[v] = g00 * gx + g01 * gy + g02 * gz;
                hy[v] = g01 * gx + g11 * gy + g12 * gz;
                hz[v] = g02 * gx + g12 * gy + g22 * gz;
            }
            const T sx = hx[0] + hx[1] + hx[2] + hx[3], sy = hy[0] + hy[1] + hy[2] + hy[3],
                    sz = hz[0] + hz[1] + hz[2] + hz[3];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                hx[v] += sx;
                hy[v] += sy;
                hz[v] += sz;
            }
#pragma unroll
            for (int i = 0; i < NL; ++i) {
                T acc_i = ys[CN.cp[t][i]];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    if (VG.D[v][0][i] != 0.0) acc_i += T(VG.D[v][0][i]) * hx[v];
                    if (VG.D[v][1][i] != 0.0) acc_i += T(VG.D[v][1][i]) * hy[v];
                    if (VG.D[v][2][i] != 0.0) acc_i += T(VG.D[v][2][i]) * hz[v];
                }
                ys[CN.cp[t][i]] = acc_i;
            }
        } else {
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
    }
#pragma unroll
    for (int j = 0; j < NCP; ++j) part[j * NT + cube] = ys[j];
    if (cube == 0) part[NCP * NT] = T(0);
    __syncthreads();
    // Closure points of the brick, each the sum of the values of the (up to 8) cubes containing it
    // in a fixed order (absent terms read a zero entry, so the sum is branch-free).  The sums are
    // formed one lane per row of points along x (interior rows, then the rows on the brick's y and
    // z faces) with the x loop unrolled, so its cube terms are compile-time constants; the rows
    // are then put back in LDS in closure order and written with consecutive lanes on
    // consecutive points: interior points to y (contiguous runs), face points to their slots.
    constexpr int QI = PB - 1, NFR = QS * QS - QI * QI;
    T rowv[2][QS];
    int rowq[2];
#pragma unroll
    for (int round = 0; round < 2; ++round) {
        const int r = threadIdx.x;
        int lb = 0, lc = 0;
        rowq[round] = -1;
        if (round == 0) {
            if (r >= QI * QI) continue;
            lb = 1 + r % QI;
            lc = 1 + r / QI;
        } else {
            if (r >= NFR) continue;
            if (r < 2 * QS) {                 // z faces: lc = 0 or PB, all lb
                lb = r % QS;
                lc = r < QS ? 0 : PB;
            } else {                          // y faces: lb = 0 or PB, lc inside
                const int u = r - 2 * QS;
                lc = 1 + u % QI;
                lb = u < QI ? 0 : PB;
            }
        }
        rowq[round] = QS * (lb + QS * lc);
        int oy[2], oz[2];
        bool vy[2], vz[2];
        axis_terms<P, B>(lb, PC, B, oy, vy);
        axis_terms<P, B>(lc, PC * PC, B * B, oz, vz);
        int oyz[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) oyz[k] = (vy[k & 1] && vz[k >> 1]) ? oy[k & 1] + oz[k >> 1] : -1;
#pragma unroll
        for (int la = 0; la < QS; ++la) {
            const int cx = la / P, ax = la % P;
            T v = T(0);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (cx < B) v += part[oyz[k] >= 0 ? oyz[k] + ax * NT + cx : ZERO];
                if (ax == 0 && cx > 0) v += part[oyz[k] >= 0 ? oyz[k] + P * NT + cx - 1 : ZERO];
            }
            rowv[round][la] = v;
        }
    }
    __syncthreads();
#pragma unroll
    for (int round = 0; round < 2; ++round)
        if (rowq[round] >= 0)
#pragma unroll
            for (int la = 0; la < QS; ++la) part[rowq[round] + la] = rowv[round][la];
    __syncthreads();
    const int64_t L = a.Lout;
    constexpr int NIN = QI * QI * QI;
    for (int r = threadIdx.x; r < NIN; r += NT) {
        const int la = 1 + r % QI, lb = 1 + (r / QI) % QI, lc = 1 + r / (QI * QI);
        const int64_t g = (bx * PB + la) + L * ((by * PB + lb) + L * (int64_t)(bz * PB + lc));
        finalize(a, g, part[la + QS * (lb + QS * lc)], false);
    }
    constexpr int NZF = 2 * QS * QS, NYF = 2 * QS * QI, NXF = 2 * QI * QI;
    for (int r = threadIdx.x; r < NZF + NYF + NXF; r += NT) {
        int la, lb, lc;
        if (r < NZF) {                       // z faces: all (la, lb)
            const int u = r % (QS * QS);
            la = u % QS;
            lb = u / QS;
            lc = r < QS * QS ? 0 : PB;
        } else if (r < NZF + NYF) {          // y faces: all la, lc inside
            const int u = (r - NZF) % (QS * QI);
            la = u % QS;
            lc = 1 + u / QS;
            lb = r - NZF < QS * QI ? 0 : PB;
        } else {                             // x faces: lb, lc inside
            const int u = (r - NZF - NYF) % (QI * QI);
            lb = 1 + u % QI;
            lc = 1 + u / QI;
            la = r - NZF - NYF < QI * QI ? 0 : PB;
        }
        put_slot<PB, T>(a, bx, by, bz, la, lb, lc, part[la + QS * (lb + QS * lc)]);
    }
}

}  // namespace fem
