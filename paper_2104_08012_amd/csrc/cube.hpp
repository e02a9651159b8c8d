// Stiffness action for P1 and P2 with one thread per cube (the cube's six tetrahedra).
//
// Same result and the same deterministic two-kernel scheme as k_brick (brick workgroups, interior
// points written directly, brick-face points through interface slots and k_fixup), organised to
// cut memory instructions, registers and LDS on gfx950's 64-wide VALU:
//  * one wave per brick of 4^3 cubes, lane = lx + 4 ly + 16 lz;
//  * the dofs of a level are numbered by their lattice point, g = I + L (J + L K) with L = p n + 1,
//    and the boundary is the lattice boundary, so no dof map is read: the wave loads the brick's
//    closure of (4p + 1)^3 values of x (boundary values as zero when columns are masked) and the
//    5^3 vertex coordinates of the brick into LDS, with consecutive lanes on consecutive points;
//  * per tetrahedron each lane reads its corners and its nodes' values from LDS at compile-time
//    offsets from one lane base, computes the geometry in FP64 from the cofactor rows
//    c1 = e2 x e3, c2 = e3 x e1, c3 = e1 x e2 of the edge vectors (J^-1 has rows c_a / det,
//    det = e1 . c1, G = |det| J^-1 J^-T = [c_a . c_b] / |det|), and accumulates the cell's
//    contributions in registers at the cube's (p+1)^3 lattice points (compile-time node-to-point
//    table, literal tabulations, zero gradient entries generate no instructions);
//  * the cubes' point values are summed across lanes in three passes with cross-lane moves (DPP
//    within a row of 16 lanes for x and y, ds_bpermute for z): after pass d, the point at local
//    index 0 along d of every cube above the first holds the sum with the cube below, so each
//    brick closure point ends in exactly one lane with the sum over the brick's cubes containing
//    it, in a fixed order (bitwise reproducible);
//  * the sums go to the LDS closure array and are written with consecutive lanes on consecutive
//    points: interior points to y (contiguous runs), brick-face points to their slots;
//  * on a refined level whose bricks each lie inside one cube of the coarsest level (GEO), the
//    geometry comes from the hierarchy's table instead: uniform refinement of the Kuhn split
//    nests every tetrahedron in one coarsest tetrahedron, on which the mesh is affine, so G of a
//    type-t tetrahedron is 2^-l times a value that depends only on the coarsest cube, the
//    coarsest tetrahedron's type t0 and t.  The wave stages its coarsest cube's 36 x 6 values in
//    LDS (scaled, in the kernel's precision) in place of the 5^3 vertex coordinates; a lane finds
//    t0 by ordering the coordinates of the tetrahedron's centroid inside the coarsest cube;
//  * loads use 32-bit offsets from uniform bases (the host keeps such levels below 4 GiB per array).
#pragma once
#include "scatter.hpp"
#include "tabulate.hpp"

namespace fem {

// 1 / d from the hardware reciprocal refined by two Newton steps r <- r + r (1 - d r) (quadratic
// convergence: well below an ulp of error left for the accuracy the kernels need).
__device__ __forceinline__ double recip(double d) {
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    e = fma(-d, r, 1.0);
    return fma(r, e, r);
}

// Order a wave's own LDS stores before its later LDS loads (a wave's LDS operations execute in
// issue order; this keeps the compiler from moving memory operations across the point).  Used
// where a wave only reads back its own region, so the other waves of the workgroup need not wait.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Cross-lane moves.  DPP row_shr:4 gives lane l the value of lane l - 4 inside its row of 16 lanes
// and the old value (zero) to the first four lanes of a row; quad_perm [0,0,1,2] gives lane l the
// value of lane l - 1 inside its quad (the first lane of a quad reads itself and is masked by the
// caller); ds_bpermute reads any lane.
template <int CTRL>
__device__ __forceinline__ int dpp32(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
    return __builtin_bit_cast(float, dpp32<CTRL>(__builtin_bit_cast(int, v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)dpp32<CTRL>((int)(uint32_t)b), hi = (uint32_t)dpp32<CTRL>((int)(uint32_t)(b >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ float lane_read(int addr, float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(addr, __builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double lane_read(int addr, double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)b);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)(b >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
// LDS offset of cube corner j (corner j at (j & 1, j >> 1 & 1, j >> 2)) in the brick's 5^3
// vertex block

template <int VS>
__host__ __device__ constexpr int vo_of(int j) {
    return (j & 1) + VS * (((j >> 1) & 1) + VS * (j >> 2));
}

// LDS layout of the brick's closure values.  Lane (lx, ly, lz) reads the points P lx + ja,
// P ly + jb, P lz + jc; for P = 2 the even and odd x coordinates are stored in two separate
// blocks with rows of 6 doubles, so a lane's base is lx + 12 ly + 108 lz and the 16 lanes of a
// row of the wave hit 16 different 8-byte bank pairs (row stride 6 -> 12 ly = 0, 12, 8, 4 mod 16).
// For P = 1 rows are padded to 6 as well.
template <int P>
struct ClosureLayout {
    static constexpr int QS = 4 * P + 1;
    static constexpr int RS = 6;                          // row stride (lb)
    static constexpr int PS = RS * QS;                    // plane stride (lc)
    static constexpr int HALF = PS * QS;                  // offset of the odd-x block (P = 2)
    static constexpr int SIZE = (P == 2 ? 2 : 1) * HALF;
    __host__ __device__ static constexpr int idx(int la, int lb, int lc) {
        return (P == 2 ? (la & 1) * HALF + (la >> 1) : la) + RS * lb + PS * lc;
    }
};

// LDS offset of cube point j = (ja, jb, jc) (ja fastest, P + 1 per axis) from the lane's base
// XL::idx(P lx, P ly, P lz): with P lx even the parity of the x coordinate is that of ja.
template <int P>
__host__ __device__ constexpr int xo_of(int j) {
    using XL = ClosureLayout<P>;
    const int ja = j % (P + 1), jb = (j / (P + 1)) % (P + 1), jc = j / ((P + 1) * (P + 1));
    return XL::idx(ja, jb, jc) - XL::idx(0, 0, 0);
}

constexpr int kQuadPrev = 0 | (0 << 2) | (1 << 4) | (2 << 6);   // quad_perm [0, 0, 1, 2]
constexpr int kRowShr4 = 0x114;                                  // row_shr:4

// Waves per SIMD the register allocation is held to (512 VGPRs per SIMD lane): what each variant
// fits without spilling, the FP64 P2 accumulators (27 doubles) being the largest live state.
template <int P, bool KVAR, typename T>
constexpr int cube_min_waves() {
    return (P == 1 || (sizeof(T) == 4 && !KVAR)) ? 4 : (sizeof(T) == 4 || !KVAR) ? 3 : 2;
}

template <int P, int B, int R, bool KVAR, bool GEO, typename T>
__global__ void __launch_bounds__(B * B * B * R, (cube_min_waves<P, KVAR, T>())) k_cube_apply(SArgs<T> a) {
    static_assert(B == 4, "one wave per brick of 4^3 cubes");
    static_assert(R == 1 || P <= 2, "bricks are merged along x for P1 and P2");
    constexpr int NL = nloc_of(P), NQ = nq_of(P, KVAR), PC = P + 1, NCP = PC * PC * PC;
    constexpr int NT = B * B * B, PB = P * B, QS = PB + 1, NQ3 = QS * QS * QS;
    constexpr int VS = B + 1, NV3 = VS * VS * VS;
    constexpr StiffTab<P, KVAR> TB{};
    constexpr CubeNodes<P> CN{};
    using XL = ClosureLayout<P>;
    constexpr int NG = 216;                                              // GEO table of a coarsest cube
    constexpr double kScale = (P == 2 && !KVAR) ? 1.0 / 120.0 : 1.0;   // P1 mass factor, vertex form
    // per wave: closure values (x on input, the brick's sums on output), the coordinates of the
    // brick's 5^3 vertices (or its coarsest cube's geometry table) and the coefficient there
    __shared__ T xcs[R][XL::SIZE];
    __shared__ double vcs[R][3][GEO ? 1 : NV3];
    __shared__ T gts[R][GEO ? NG : 1];
    __shared__ T kls[R][KVAR ? NV3 : 1];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / NT), lane = threadIdx.x % NT;
    T* __restrict__ xc = xcs[wave];
    double(*__restrict__ vc)[GEO ? 1 : NV3] = vcs[wave];
    T* __restrict__ gt = gts[wave];
    T* __restrict__ kl = kls[wave];
    // workgroup = R bricks along x (wave w: brick R px + w)
    const int pid = brick_of_block(blockIdx.x, gridDim.x);
    const int nb = a.nb, nbx = a.nbx;
    const int px = pid % nbx, by = (pid / nbx) % nb, bz = pid / (nbx * nb);
    const int bx = px * R + wave;
    const int lx = lane % B, ly = (lane / B) % B, lz = lane / (B * B);
    const uint32_t Lo = (uint32_t)a.Lout;

    // ---- stage the brick's closure values of x and its vertex data in LDS ----
    // (all loads are issued before the first LDS store; indices past the end are clamped)
    const uint32_t gb = (uint32_t)(bx * PB) + Lo * ((uint32_t)(by * PB) + Lo * (uint32_t)(bz * PB));
    {
        // P2: part A, lanes (la, lb) = (lane % 9, lane / 9) for lb < 7, every plane lc; part B,
        // lanes (la, lb, lc0) with lb = 7, 8 and lc = lc0 + 3 it.  A plane's offset is uniform,
        // so the loads and LDS stores need no per-load address arithmetic.  P1: flat.
        constexpr int NIT = P == 2 ? QS + 3 : (NQ3 + NT - 1) / NT;
        T v[NIT];
        int li[NIT];
        const uint32_t LL = Lo * Lo;
        const int la = lane % QS, rA = lane / QS, rB = rA < 5 ? rA : 5;
        const int lbB = 7 + rB % 2, lc0 = rB / 2;
        if constexpr (P == 2) {
            const uint32_t oA = gb + (uint32_t)la + Lo * (uint32_t)rA;
            const uint32_t oB = gb + (uint32_t)la + Lo * (uint32_t)lbB + LL * (uint32_t)lc0;
#pragma unroll
            for (int lc = 0; lc < QS; ++lc) v[lc] = ldg(a.x + (size_t)lc * LL, oA);
#pragma unroll
            for (int it = 0; it < 3; ++it) v[QS + it] = ldg(a.x + (size_t)(3 * it) * LL, oB);
        } else {
#pragma unroll
            for (int it = 0; it < NIT; ++it) {
                const int r = (lane + NT * it < NQ3) ? lane + NT * it : NQ3 - 1;
                const int ra = r % QS, q = r / QS, rb = q % QS, rc = q / QS;
                v[it] = ldg(a.x, gb + (uint32_t)ra + Lo * ((uint32_t)rb + Lo * (uint32_t)rc));
                li[it] = XL::idx(ra, rb, rc);
            }
        }
        const uint32_t n1 = (uint32_t)a.n + 1, NV = a.nv;
        const uint32_t vb = (uint32_t)(bx * B) + n1 * ((uint32_t)(by * B) + n1 * (uint32_t)(bz * B));
        constexpr int NVIT = (NV3 + NT - 1) / NT, NGIT = (NG + NT - 1) / NT;
        double cx[NVIT], cy[NVIT], cz[NVIT], gv[NGIT];
        T kv[NVIT];
#pragma unroll
        for (int it = 0; it < NVIT; ++it) {
            const int r = (lane + NT * it < NV3) ? lane + NT * it : NV3 - 1;
            const uint32_t w = vb + (uint32_t)(r % VS) + n1 * ((uint32_t)((r / VS) % VS) + n1 * (uint32_t)(r / (VS * VS)));
            if constexpr (!GEO) {
                cx[it] = ldg(a.vxyz, w);
                cy[it] = ldg(a.vxyz, NV + w);
                cz[it] = ldg(a.vxyz, 2 * NV + w);
            }
            if constexpr (KVAR) kv[it] = ldg(a.k, w);
        }
        if constexpr (GEO) {
            // the brick's coarsest cube (the brick lies inside it: 2^geo_shift >= B)
            const int sh = a.geo_shift;
            const uint32_t n0 = (uint32_t)a.n >> sh;
            const uint32_t q0 = (uint32_t)((bx * B) >> sh) + n0 * ((uint32_t)((by * B) >> sh) + n0 * (uint32_t)((bz * B) >> sh));
#pragma unroll
            for (int it = 0; it < NGIT; ++it) {
                const int r = (lane + NT * it < NG) ? lane + NT * it : NG - 1;
                gv[it] = ldg(a.geo, q0 * (uint32_t)NG + (uint32_t)r);
            }
        }
        if constexpr (P == 2) {
            const int iA = XL::idx(la, rA, 0), iB = XL::idx(la, lbB, lc0);
            if (lane < 7 * QS)
#pragma unroll
                for (int lc = 0; lc < QS; ++lc) xc[iA + XL::PS * lc] = v[lc];
            if (lane < 6 * QS)
#pragma unroll
                for (int it = 0; it < 3; ++it) xc[iB + 3 * XL::PS * it] = v[QS + it];
        } else {
#pragma unroll
            for (int it = 0; it < NIT; ++it)
                if (lane + NT * it < NQ3) xc[li[it]] = v[it];
        }
#pragma unroll
        for (int it = 0; it < NVIT; ++it) {
            const int r = lane + NT * it;
            if (r < NV3) {
                if constexpr (!GEO) {
                    vc[0][r] = cx[it];
                    vc[1][r] = cy[it];
                    vc[2][r] = cz[it];
                }
                if constexpr (KVAR) kl[r] = kv[it];
            }
        }
        if constexpr (GEO) {
            const double gs = a.geo_scale * kScale;
#pragma unroll
            for (int it = 0; it < NGIT; ++it) {
                const int r = lane + NT * it;
                if (r < NG) gt[r] = T(gv[it] * gs);
            }
        }
        // masked columns: zero the closure faces that lie on the domain boundary
        if (a.mask_cols && (bx == 0 || by == 0 || bz == 0 || bx == nb - 1 || by == nb - 1 || bz == nb - 1)) {
#pragma unroll
            for (int f = 0; f < 6; ++f) {
                const int d = f >> 1, hi = f & 1;
                const int bd = d == 0 ? bx : d == 1 ? by : bz;
                if (bd != (hi ? nb - 1 : 0)) continue;
                for (int r = lane; r < QS * QS; r += NT) {
                    const int u = r % QS, w = r / QS, e = hi ? PB : 0;
                    xc[d == 0 ? XL::idx(e, u, w) : d == 1 ? XL::idx(u, e, w) : XL::idx(u, w, e)] = T(0);
                }
            }
        }
    }
    wave_sync();   // each wave reads back only its own staged data

    // ---- the six tetrahedra of the lane's cube ----
    const int xb = XL::idx(P * lx, P * ly, P * lz);       // LDS index of the cube's point 0
    const int vbl = lx + VS * (ly + VS * lz);              // vertex index of the cube's corner 0
    // GEO: 4 x the cube's position inside its coarsest cube
    const int gmask = GEO ? (1 << a.geo_shift) - 1 : 0;
    const int ax4 = 4 * ((bx * B + lx) & gmask), ay4 = 4 * ((by * B + ly) & gmask), az4 = 4 * ((bz * B + lz) & gmask);
    T ys[NCP];
#pragma unroll
    for (int j = 0; j < NCP; ++j) ys[j] = T(0);
#pragma unroll
    for (int t = 0; t < 6; ++t) {
        // keep the LDS reads inside each tetrahedron, so they are not held in registers across it
        __asm__ volatile("" ::: "memory");
        // path tetrahedron: v0 = corner 0, v1 = e_s0, v2 = e_s0 + e_s1, v3 = corner 7 (corner j
        // at offset (j & 1, j >> 1 & 1, j >> 2))
        const int s0 = perm_axis(t, 0), s1 = perm_axis(t, 1);
        const int j1 = 1 << s0, j2 = (1 << s0) | (1 << s1);
        T gm[6];                                 // G: 00, 11, 22, 01, 02, 12
        double c1x = 0, c1y = 0, c1z = 0, c2x = 0, c2y = 0, c2z = 0, c3x = 0, c3y = 0, c3z = 0, inv = 0;
        if constexpr (GEO) {
            const int ux = ax4 + centroid4(t, 0), uy = ay4 + centroid4(t, 1), uz = az4 + centroid4(t, 2);
            const int t0 = (kPathTypeCode >> (3 * ((ux > uy) + 2 * (ux > uz) + 4 * (uy > uz)))) & 7;
            const int g0 = 6 * (6 * t0 + t);
#pragma unroll
            for (int e = 0; e < 6; ++e) gm[e] = gt[g0 + e];
        } else {
            double e1[3], e2[3], e3[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double p0 = vc[d][vbl];
                e1[d] = vc[d][vbl + vo_of<VS>(j1)] - p0;
                e2[d] = vc[d][vbl + vo_of<VS>(j2)] - p0;
                e3[d] = vc[d][vbl + vo_of<VS>(7)] - p0;
            }
            c1x = e2[1] * e3[2] - e2[2] * e3[1], c1y = e2[2] * e3[0] - e2[0] * e3[2], c1z = e2[0] * e3[1] - e2[1] * e3[0];
            c2x = e3[1] * e1[2] - e3[2] * e1[1], c2y = e3[2] * e1[0] - e3[0] * e1[2], c2z = e3[0] * e1[1] - e3[1] * e1[0];
            c3x = e1[1] * e2[2] - e1[2] * e2[1], c3y = e1[2] * e2[0] - e1[0] * e2[2], c3z = e1[0] * e2[1] - e1[1] * e2[0];
            const double det = e1[0] * c1x + e1[1] * c1y + e1[2] * c1z;
            inv = kScale * recip(fabs(det));
            if constexpr (P == 2) {
                gm[0] = T((c1x * c1x + c1y * c1y + c1z * c1z) * inv);
                gm[1] = T((c2x * c2x + c2y * c2y + c2z * c2z) * inv);
                gm[2] = T((c3x * c3x + c3y * c3y + c3z * c3z) * inv);
                gm[3] = T((c1x * c2x + c1y * c2y + c1z * c2z) * inv);
                gm[4] = T((c1x * c3x + c1y * c3y + c1z * c3z) * inv);
                gm[5] = T((c2x * c3x + c2y * c3y + c2z * c3z) * inv);
            } else {
#pragma unroll
                for (int e = 0; e < 6; ++e) gm[e] = T(0);
            }
        }
        const T g00 = gm[0], g11 = gm[1], g22 = gm[2], g01 = gm[3], g02 = gm[4], g12 = gm[5];
        // the cell's nodal values, read once the geometry is done (fewer values live at once)
        __asm__ volatile("" ::: "memory");
        T xs[NL];
#pragma unroll
        for (int i = 0; i < NL; ++i) xs[i] = xc[xb + xo_of<P>(CN.cp[t][i])];
        T kt[4];
        if constexpr (KVAR) {
            kt[0] = kl[vbl];
            kt[1] = kl[vbl + vo_of<VS>(j1)];
            kt[2] = kl[vbl + vo_of<VS>(j2)];
            kt[3] = kl[vbl + vo_of<VS>(7)];
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
                    if (VG.D[v][0][i] != 0.0) gx += T(VG.D[v][0][i]) * xs[i];
                    if (VG.D[v][1][i] != 0.0) gy += T(VG.D[v][1][i]) * xs[i];
                    if (VG.D[v][2][i] != 0.0) gz += T(VG.D[v][2][i]) * xs[i];
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
        } else if constexpr (P == 1) {
            // one point (the gradient is constant): G g = C (C^T g) / |det| with C the cofactor
            // rows, cheaper than forming G (21 instead of 33 multiply-adds)
            constexpr int q = 0;
            T gx = T(0), gy = T(0), gz = T(0);
#pragma unroll
            for (int i = 0; i < NL; ++i) {
                if (TB.D[q][0][i] != 0.0) gx += T(TB.D[q][0][i]) * xs[i];
                if (TB.D[q][1][i] != 0.0) gy += T(TB.D[q][1][i]) * xs[i];
                if (TB.D[q][2][i] != 0.0) gz += T(TB.D[q][2][i]) * xs[i];
            }
            T s = T(TB.w[q]);
            if constexpr (KVAR)
                s *= T(TB.lam[q][0]) * kt[0] + T(TB.lam[q][1]) * kt[1] + T(TB.lam[q][2]) * kt[2] +
                     T(TB.lam[q][3]) * kt[3];
            T wx, wy, wz;
            if constexpr (GEO) {
                wx = s * (g00 * gx + g01 * gy + g02 * gz);
                wy = s * (g01 * gx + g11 * gy + g12 * gz);
                wz = s * (g02 * gx + g12 * gy + g22 * gz);
            } else {
                const T a1x = T(c1x), a1y = T(c1y), a1z = T(c1z), a2x = T(c2x), a2y = T(c2y), a2z = T(c2z),
                        a3x = T(c3x), a3y = T(c3y), a3z = T(c3z);
                const T vx = gx * a1x + gy * a2x + gz * a3x;
                const T vy = gx * a1y + gy * a2y + gz * a3y;
                const T vz = gx * a1z + gy * a2z + gz * a3z;
                const T sc = s * T(inv);
                wx = sc * (a1x * vx + a1y * vy + a1z * vz);
                wy = sc * (a2x * vx + a2y * vy + a2z * vz);
                wz = sc * (a3x * vx + a3y * vy + a3z * vz);
            }
#pragma unroll
            for (int i = 0; i < NL; ++i) {
                T acc_i = ys[CN.cp[t][i]];
                if (TB.D[q][0][i] != 0.0) acc_i += T(TB.D[q][0][i]) * wx;
                if (TB.D[q][1][i] != 0.0) acc_i += T(TB.D[q][1][i]) * wy;
                if (TB.D[q][2][i] != 0.0) acc_i += T(TB.D[q][2][i]) * wz;
                ys[CN.cp[t][i]] = acc_i;
            }
        } else {
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

    // ---- sums over the brick's cubes, one axis at a time ----
    // x: point (0, b, c) of cube lx > 0 adds point (P, b, c) of cube lx - 1
#pragma unroll
    for (int j = 0; j < PC * PC; ++j) {
        const T v = dpp_move<kQuadPrev>(ys[P + PC * j]);
        ys[PC * j] += (lx == 0) ? T(0) : v;
    }
    // y: point (a, 0, c) of cube ly > 0 adds point (a, P, c) of cube ly - 1 (lanes with ly = 0
    // receive zero from the row shift)
#pragma unroll
    for (int c = 0; c < PC; ++c)
#pragma unroll
        for (int a0 = 0; a0 < PC; ++a0) ys[a0 + PC * PC * c] += dpp_move<kRowShr4>(ys[a0 + PC * (P + PC * c)]);
    // z: point (a, b, 0) of cube lz > 0 adds point (a, b, P) of cube lz - 1
    {
        const int addr = 4 * (lz == 0 ? lane : lane - B * B);
#pragma unroll
        for (int j = 0; j < PC * PC; ++j) {
            const T v = lane_read(addr, ys[j + PC * PC * P]);
            ys[j] += (lz == 0) ? T(0) : v;
        }
    }
    // Each closure point (la, lb, lc) of the brick is now held by the cube min(la / P, B - 1)
    // (and likewise in y, z) at local index la - P * that cube.
    wave_sync();   // the held points overwrite this wave's own closure values
#pragma unroll
    for (int j = 0; j < NCP; ++j) {
        const int ja = j % PC, jb = (j / PC) % PC, jc = j / (PC * PC);
        if ((ja < P || lx == B - 1) && (jb < P || ly == B - 1) && (jc < P || lz == B - 1))
            xc[xb + xo_of<P>(j)] = ys[j];
    }
    __syncthreads();   // the exchange reads the neighbouring wave's closure

    // ---- write-out: interior points to y, face points to their slots ----
    constexpr int QI = PB - 1, NIN = QI * QI * QI, PBX = R * PB;
    const T alpha = a.alpha, beta = a.beta;
    const uint32_t nbu = (uint32_t)nb, nbxu = (uint32_t)nbx, npx = Lo - nbxu - 1, tot = a.if_tot;
    T* __restrict__ slots = a.slots;
    if constexpr (P == 2) {
        // x faces shared by the workgroup's bricks: wave w > 0 adds the upper x face of wave w - 1
        // (lower brick first) to its own lower x face, which is then complete and written to y
        // as part of the interior; wave w < R - 1 leaves its upper x face to wave w + 1
        if constexpr (R > 1) {
            if (wave > 0) {
                const T* __restrict__ xp = xcs[wave - 1];
                for (int r = lane; r < QS * QS; r += NT) {
                    const int lb = r % QS, lc = r / QS;
                    const int i = XL::idx(0, lb, lc);
                    xc[i] = xp[XL::idx(PB, lb, lc)] + xc[i];
                }
            }
        }
        // lane tiles whose per-iteration offsets are uniform (plane, face) or compile-time (LDS);
        // la runs over [la_lo, PB - 1]: la = 0 is a workgroup face only for wave 0
        const int la_lo = wave == 0 ? 1 : 0;
        const uint32_t LL = Lo * Lo;
        const uint32_t LA0 = (uint32_t)(wave * PB);   // workgroup-local x of the brick's la = 0
        {   // interior: lanes (la, lb) = (lane % 8, 1 + lane / 8), lb <= 7, planes lc = 1..7
            const int la = lane % PB, lb = 1 + lane / PB;
            const uint32_t o = gb + (uint32_t)la + Lo * (uint32_t)lb;
            const int i0 = XL::idx(la, lb, 0);
            if (lb <= QI && la >= la_lo)
#pragma unroll
                for (int lc = 1; lc <= QI; ++lc) {
                    T v = alpha * xc[i0 + XL::PS * lc];
                    if (beta != T(0)) v += beta * ldg(a.z + (size_t)lc * LL, o);
                    *reinterpret_cast<T*>(reinterpret_cast<char*>(a.y + (size_t)lc * LL) + o * (uint32_t)sizeof(T)) = v;
                }
        }
        {   // workgroup x faces (wave 0: la = 0; wave R - 1: la = PB): lanes (lb, c) = (lane % 9,
            // lane / 9), lc = c + 7 blk
            const int lb = lane % QS, c = lane / QS;
            const uint32_t o = (uint32_t)lb + Lo * (uint32_t)c;
#pragma unroll
            for (int sd = 0; sd < 2; ++sd) {
                if (sd == 0 ? wave != 0 : wave != R - 1) continue;
#pragma unroll
                for (int blk = 0; blk < 2; ++blk) {
                    if (lane < 7 * QS && (blk == 0 || c < 2)) {
                        const uint32_t code = (sd == 0 ? 1u : 0u) | (lb == 0 ? 2u : 0u) | (blk == 0 && c == 0 ? 4u : 0u);
                        const uint32_t t = iface_x0<PBX, PB>(px, by, bz, sd, Lo) + 7 * blk * Lo + o;
                        slots[(size_t)code * tot + t] = xc[XL::idx(sd * PB, lb, c) + 7 * blk * XL::PS];
                    }
                }
            }
        }
        {   // y faces (lb = 0, PB): lanes (la, lc) = (lane % 8, lane / 8) for lc <= 7, then lc = 8
            const int la = lane % PB, lc = lane / PB;
            const uint32_t o = LA0 + (uint32_t)la + npx * (uint32_t)lc;
            const int i0 = XL::idx(la, 0, lc);
            const uint32_t code = lc == 0 ? 4u : 0u;
            if (la >= la_lo) {
#pragma unroll
                for (int sd = 0; sd < 2; ++sd) {
                    const uint32_t ty = iface_y0<PBX, PB>(px, by, bz, sd, Lo, nbxu, a.if_c0);
                    slots[(size_t)(code | (sd == 0 ? 2u : 0u)) * tot + ty + o] = xc[i0 + XL::RS * PB * sd];
                    if (lane < PB)   // lc = PB
                        slots[(size_t)(sd == 0 ? 2u : 0u) * tot + ty + o + npx * PB] =
                            xc[i0 + XL::RS * PB * sd + XL::PS * PB];
                }
            }
        }
        {   // z faces (lc = 0, PB): lanes (la, lb) = (lane % 8, 1 + lane / 8), lb <= 7
            const int la = lane % PB, lb = 1 + lane / PB;
            const uint32_t o = LA0 + (uint32_t)la + npx * (uint32_t)lb;
            const int i0 = XL::idx(la, lb, 0);
            if (lb <= QI && la >= la_lo)
#pragma unroll
                for (int sd = 0; sd < 2; ++sd) {
                    const uint32_t t = iface_z0<PBX, PB>(px, by, bz, sd, Lo, nbxu, nbu, a.if_c01) + o;
                    slots[(size_t)(sd == 0 ? 4u : 0u) * tot + t] = xc[i0 + XL::PS * PB * sd];
                }
        }
    } else {
        // x faces shared by the workgroup's bricks, as for P2: wave w > 0 adds the upper x face of
        // wave w - 1 to its own lower x face and writes it to y with its interior; the x position
        // of a brick point in the workgroup is w PB + la
        if constexpr (R > 1) {
            if (wave > 0) {
                const T* __restrict__ xp = xcs[wave - 1];
                for (int r = lane; r < QS * QS; r += NT) {
                    const int lb = r % QS, lc = r / QS;
                    const int i = XL::idx(0, lb, lc);
                    xc[i] = xp[XL::idx(PB, lb, lc)] + xc[i];
                }
            }
        }
        const int la_lo = wave == 0 ? 1 : 0;
        const uint32_t LA0 = (uint32_t)(wave * PB);
#pragma unroll
        for (int it = 0; it < (PB * QI * QI + NT - 1) / NT; ++it) {   // interior: la in [la_lo, PB - 1]
            const int r = lane + NT * it;
            const int la = r % PB, q = r / PB, lb = 1 + q % QI, lc = 1 + q / QI;
            if (r < PB * QI * QI && la >= la_lo) {
                const uint32_t g = gb + (uint32_t)la + Lo * ((uint32_t)lb + Lo * (uint32_t)lc);
                T v = alpha * xc[XL::idx(la, lb, lc)];
                if (beta != T(0)) v += beta * ldg(a.z, g);
                *reinterpret_cast<T*>(reinterpret_cast<char*>(a.y) + g * (uint32_t)sizeof(T)) = v;
            }
        }
        // Face points, one face family at a time (the slot index is affine within a face); the
        // slot plane is code = [la == 0] + 2 [lb == 0] + 4 [lc == 0].
        for (int r = lane; r < 2 * QS * QS; r += NT) {                 // workgroup x faces
            const int sd = r / (QS * QS), u = r % (QS * QS), lb = u % QS, lc = u / QS, la = sd * PB;
            if (sd == 0 ? wave != 0 : wave != R - 1) continue;
            const uint32_t t = iface_x0<PBX, PB>(px, by, bz, sd, Lo) + (uint32_t)lb + Lo * (uint32_t)lc;
            const uint32_t code = (sd == 0 ? 1u : 0u) | (lb == 0 ? 2u : 0u) | (lc == 0 ? 4u : 0u);
            slots[(size_t)code * tot + t] = xc[XL::idx(la, lb, lc)];
        }
        for (int r = lane; r < 2 * PB * QS; r += NT) {                 // y faces: lb = 0, PB
            const int sd = r / (PB * QS), u = r % (PB * QS), la = u % PB, lc = u / PB, lb = sd * PB;
            if (la < la_lo) continue;
            const uint32_t t = iface_y0<PBX, PB>(px, by, bz, sd, Lo, nbxu, a.if_c0) + LA0 + (uint32_t)la + npx * (uint32_t)lc;
            const uint32_t code = (sd == 0 ? 2u : 0u) | (lc == 0 ? 4u : 0u);
            slots[(size_t)code * tot + t] = xc[XL::idx(la, lb, lc)];
        }
        for (int r = lane; r < 2 * PB * QI; r += NT) {                 // z faces: lc = 0, PB; lb inside
            const int sd = r / (PB * QI), u = r % (PB * QI), la = u % PB, lb = 1 + u / PB, lc = sd * PB;
            if (la < la_lo) continue;
            const uint32_t t = iface_z0<PBX, PB>(px, by, bz, sd, Lo, nbxu, nbu, a.if_c01) + LA0 + (uint32_t)la + npx * (uint32_t)lb;
            const uint32_t code = sd == 0 ? 4u : 0u;
            slots[(size_t)code * tot + t] = xc[XL::idx(la, lb, lc)];
        }
    }
}

}  // namespace fem
