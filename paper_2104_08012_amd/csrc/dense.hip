// Dense inverse of the coarsest level's interior operator block (SPD, at most 40000 rows), for the
// exact FP64 coarse-grid solve that replaces the paper's direct (LU) coarse solver (Section 4).
//
// Blocked Gauss-Jordan sweep.  Sweeping the index block K of the current matrix M maps
//   M_KK -> P = M_KK^-1,  M_KJ -> P M_KJ,  M_IK -> -M_IK P,  M_IJ -> M_IJ - M_IK P M_KJ   (I, J outside K),
// and once every block has been swept M = A^-1.  No pivoting: the diagonal blocks of the Schur
// complements of an SPD matrix are SPD.
//
// Only the lower triangle is kept.  With the blocks swept in order (rows above K swept, rows
// below not), a partially swept symmetric matrix has m_ij = m_ji where i and j are both swept or
// both not, and m_ij = -m_ji otherwise.  So with W the current column panel M_:K (rows below K:
// the stored M_IK; rows above: -M_KI^T) and Vs_J = s_J W_J P (s_J = -1 above K, +1 below):
//   M_IJ -= W_I Vs_J^T on the lower tiles outside K      (n^3 flops in all, half of the full sweep),
//   M_IK = -Vs_I below K,  M_KJ = Vs_J^T left of K,  M_KK = P.
// Pivot blocks of 256 make the trailing update a rank-256 product on the FP64 matrix cores,
// bound by arithmetic rather than by re-reading the matrix (12.8 GB at 40000 rows) once per
// block.  P is the inverse of a dense copy of M_KK by the full sweep with 64-wide blocks, each
// 64 x 64 pivot inverted by one workgroup with the block in registers.
#include "vec.hpp"

namespace fem {

namespace {

constexpr int DB = 256;   // pivot block of the outer sweep
constexpr int SB = 64;    // pivot block of the sweep on a diagonal block (and tile of the panel kernels)

// Invert the b x b block at (k0, k0) of a matrix with leading dimension ld in place (Gauss-Jordan,
// b <= 64).  One workgroup; the block, padded to 64 x 64 with the identity (which the sweep leaves
// as it is), stays in registers: thread t holds column t % 64 of rows t / 64 + 4 m, m = 0..15.  At
// step k the current row k and column k are published in LDS (two alternating buffers, so one
// barrier per step).
__global__ void __launch_bounds__(256) k_gj_pivot(int64_t ld, int64_t k0, int b, double* A) {
    __shared__ double row[2][SB], col[2][SB];
    const int j = threadIdx.x % SB, i0 = threadIdx.x / SB;
    double v[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        const int i = i0 + 4 * m;
        v[m] = (i < b && j < b) ? A[(k0 + i) * ld + k0 + j] : (i == j ? 1.0 : 0.0);
    }
#pragma unroll
    for (int k = 0; k < SB; ++k) {
        const int h = k & 1, mk = k >> 2;
        if (i0 == (k & 3)) row[h][j] = v[mk];
        if (j == k)
#pragma unroll
            for (int m = 0; m < 16; ++m) col[h][i0 + 4 * m] = v[m];
        __syncthreads();
        const double piv = 1.0 / row[h][k];
        const double rj = row[h][j];
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const int i = i0 + 4 * m;
            const double ci = col[h][i];
            if (i == k) v[m] = (j == k) ? piv : rj * piv;
            else if (j == k) v[m] = -ci * piv;
            else v[m] -= ci * rj * piv;
        }
    }
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        const int i = i0 + 4 * m;
        if (i < b && j < b) A[(k0 + i) * ld + k0 + j] = v[m];
    }
}

// Tiled FP64 GEMM  C = alpha A B + beta C  (row-major, leading dimensions lda/ldb/ldc), 64 x 64
// tiles of C per workgroup, 4 x 4 register blocks per thread, K in chunks of 16 staged in LDS.
// Rows of C in [rskip_lo, rskip_hi) and columns in [cskip_lo, cskip_hi) are left untouched.  Every
// workgroup reads all of its A and B inputs before writing its C tile, so the 64-wide sweep on a
// diagonal block can run in place: its row panel (one tile row) writes the rows it reads, each
// tile only its own columns; its column panel (one tile column) the columns it reads, each tile
// only its own rows; its trailing update never writes the pivot rows or columns it reads.
constexpr int GT = 64, GK = 16;

__global__ void __launch_bounds__(256) k_gemm(int64_t M, int64_t N, int K, double alpha, const double* A, int64_t lda,
                                              const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
                                              int64_t rskip_lo, int64_t rskip_hi, int64_t cskip_lo, int64_t cskip_hi) {
    const int64_t i0 = (int64_t)blockIdx.y * GT, j0 = (int64_t)blockIdx.x * GT;
    __shared__ double As[GK][GT + 1];
    __shared__ double Bs[GK][GT + 1];
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    double acc[4][4] = {};
    for (int kk = 0; kk < K; kk += GK) {
        for (int e = threadIdx.x; e < GK * GT; e += 256) {
            const int r = e / GK, c = e % GK;
            const int64_t gi = i0 + r;
            As[c][r] = (gi < M && kk + c < K) ? A[gi * lda + kk + c] : 0.0;
            const int rr = e / GT, cc = e % GT;
            const int64_t gj = j0 + cc;
            Bs[rr][cc] = (gj < N && kk + rr < K) ? B[(int64_t)(kk + rr) * ldb + gj] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < GK; ++c) {
            double a[4], bb[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = As[c][ty * 4 + u];
                bb[u] = Bs[c][tx * 4 + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * bb[v];
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t gi = i0 + ty * 4 + u;
        if (gi >= M || (gi >= rskip_lo && gi < rskip_hi)) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t gj = j0 + tx * 4 + v;
            if (gj >= N || (gj >= cskip_lo && gj < cskip_hi)) continue;
            double* c = &C[gi * ldc + gj];
            *c = (beta == 0.0) ? alpha * acc[u][v] : alpha * acc[u][v] + beta * *c;
        }
    }
}

// W (n x b, row-major): the column panel of block K = [k0, k0 + b) read from the lower triangle.
// Tile (64 rows from i0, 64 panel columns from c0) per workgroup; rows above K are read along rows
// of the panel's transpose (coalesced) and transposed through LDS; rows inside K are zeroed.
__global__ void __launch_bounds__(256) k_gj_gather(int64_t n, int b, int64_t k0, const double* __restrict__ A,
                                                   double* __restrict__ W) {
    __shared__ double t[SB][SB + 1];
    const int64_t i0 = (int64_t)blockIdx.x * SB;
    const int c0 = blockIdx.y * SB;
    if (i0 >= k0 && i0 < k0 + b) {
        for (int e = threadIdx.x; e < SB * SB; e += 256) {
            const int64_t i = i0 + e / SB;
            const int c = c0 + e % SB;
            if (i < n && c < b) W[i * b + c] = 0.0;
        }
        return;
    }
    if (i0 >= k0 + b) {
        for (int e = threadIdx.x; e < SB * SB; e += 256) {
            const int64_t i = i0 + e / SB;
            const int c = c0 + e % SB;
            if (i < n && c < b) W[i * b + c] = A[i * n + k0 + c];
        }
        return;
    }
    for (int e = threadIdx.x; e < SB * SB; e += 256) {
        const int c = e / SB, r = e % SB;
        if (c0 + c < b && i0 + r < n) t[c][r] = -A[(k0 + c0 + c) * n + i0 + r];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < SB * SB; e += 256) {
        const int r = e / SB, c = e % SB;
        if (c0 + c < b && i0 + r < n) W[(i0 + r) * b + c0 + c] = t[c][r];
    }
}

// Pb (b x b): dense symmetric copy of the diagonal block K from its lower 64 x 64 tiles.
__global__ void __launch_bounds__(256) k_gj_block(int64_t n, int b, int64_t k0, const double* __restrict__ A,
                                                  double* __restrict__ Pb) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= b * b) return;
    const int r = e / b, c = e % b;
    Pb[e] = (r / SB >= c / SB) ? A[(k0 + r) * n + k0 + c] : A[(k0 + c) * n + k0 + r];
}

// Lower tile t = I (I + 1) / 2 + J, I >= J, of a tile grid.
__device__ __forceinline__ void lower_tile(int64_t t, int& I, int& J) {
    int i = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((int64_t)(i + 1) * (i + 2) / 2 <= t) ++i;
    while ((int64_t)i * (i + 1) / 2 > t) --i;
    I = i;
    J = (int)(t - (int64_t)i * (i + 1) / 2);
}

// Trailing update M_IJ -= W_I Vs_J^T on the lower 128 x 128 tiles outside K, on the FP64 matrix
// cores (v_mfma_f64_16x16x4_f64: D = A B + C with A 16 x 4, B 4 x 16; lane l holds A[l % 16][l / 16]
// and B[l / 16][l % 16], and D[l / 16 + 4 r][l % 16] in accumulator entry r).  Wave w of the
// four computes the 64 x 64 quarter (w / 2, w % 2) of the tile as 4 x 4 blocks of 16 x 16; the
// rank-b product runs over chunks of 16 panel columns staged in LDS row-major (the next chunk is
// loaded into registers while the current one is multiplied).  Tiles that meet K (whole tiles:
// k0 and k0 + b are multiples of 128, or k0 + b = n) return at once.
typedef double dx4 __attribute__((ext_vector_type(4)));
constexpr int UT = 128, UK = 16, ULD = UK + 1;

__global__ void __launch_bounds__(256, 2) k_gj_update(int64_t n, int b, int64_t k0, const double* __restrict__ W,
                                                   const double* __restrict__ Vs, double* __restrict__ A) {
    int I, J;
    lower_tile(blockIdx.x, I, J);
    const int64_t i0 = (int64_t)I * UT, j0 = (int64_t)J * UT, k1 = k0 + b;
    if ((i0 < k1 && i0 + UT > k0) || (j0 < k1 && j0 + UT > k0)) return;
    __shared__ double As[UT * ULD];
    __shared__ double Bs[UT * ULD];
    const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
    const int wr = wave / 2, wc = wave % 2, li = lane % 16, lk = lane / 16;
    const int sr = tid / UK, sc = tid % UK;   // staging: rows sr + 16 q, panel column sc
    dx4 acc[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = dx4{0.0, 0.0, 0.0, 0.0};
    double wa[8], wb[8];
    {
        const bool in = sc < b;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t ri = i0 + sr + 16 * q, rj = j0 + sr + 16 * q;
            wa[q] = (in && ri < n) ? W[ri * b + sc] : 0.0;
            wb[q] = (in && rj < n) ? Vs[rj * b + sc] : 0.0;
        }
    }
    for (int kk = 0; kk < b; kk += UK) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            As[(sr + 16 * q) * ULD + sc] = wa[q];
            Bs[(sr + 16 * q) * ULD + sc] = wb[q];
        }
        __syncthreads();
        const int kn = kk + UK;
        if (kn < b) {
            const bool in = kn + sc < b;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int64_t ri = i0 + sr + 16 * q, rj = j0 + sr + 16 * q;
                wa[q] = (in && ri < n) ? W[ri * b + kn + sc] : 0.0;
                wb[q] = (in && rj < n) ? Vs[rj * b + kn + sc] : 0.0;
            }
        }
#pragma unroll
        for (int ks = 0; ks < UK; ks += 4) {
            double a[4], bb[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = As[(64 * wr + 16 * u + li) * ULD + ks + lk];
                bb[u] = Bs[(64 * wc + 16 * u + li) * ULD + ks + lk];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], bb[v], acc[u][v], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t i = i0 + 64 * wr + 16 * u + lk + 4 * r;
            if (i >= n) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t j = j0 + 64 * wc + 16 * v + li;
                if (j < n) A[i * n + j] -= acc[u][v][r];
            }
        }
}

// The swept panels and pivot block, tile (64 rows of Vs from i0, 64 panel columns from c0) per
// workgroup: rows below K give M_IK = -Vs_I, rows above K give M_KI = Vs_I^T (transposed through
// LDS, written along rows of M), rows inside K copy P into M_KK.
__global__ void __launch_bounds__(256) k_gj_panels(int64_t n, int b, int64_t k0, const double* __restrict__ Vs,
                                                   const double* __restrict__ Pb, double* __restrict__ A) {
    __shared__ double t[SB][SB + 1];
    const int64_t i0 = (int64_t)blockIdx.x * SB;
    const int c0 = blockIdx.y * SB;
    if (i0 >= k0 && i0 < k0 + b) {
        for (int e = threadIdx.x; e < SB * SB; e += 256) {
            const int64_t i = i0 + e / SB;
            const int c = c0 + e % SB;
            if (i < n && c < b) A[i * n + k0 + c] = Pb[(i - k0) * b + c];
        }
        return;
    }
    if (i0 >= k0 + b) {
        for (int e = threadIdx.x; e < SB * SB; e += 256) {
            const int64_t i = i0 + e / SB;
            const int c = c0 + e % SB;
            if (i < n && c < b) A[i * n + k0 + c] = -Vs[i * b + c];
        }
        return;
    }
    for (int e = threadIdx.x; e < SB * SB; e += 256) {
        const int r = e / SB, c = e % SB;
        if (c0 + c < b && i0 + r < n) t[c][r] = Vs[(i0 + r) * b + c0 + c];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < SB * SB; e += 256) {
        const int c = e / SB, r = e % SB;
        if (c0 + c < b && i0 + r < n) A[(k0 + c0 + c) * n + i0 + r] = t[c][r];
    }
}

// In-place inverse of a dense b x b SPD matrix (leading dimension ld) by the full Gauss-Jordan
// sweep with 64-wide pivot blocks.
void invert_block(int b, int64_t ld, double* A, hipStream_t s) {
    const unsigned tn = (unsigned)((b + GT - 1) / GT);
    for (int64_t k0 = 0; k0 < b; k0 += SB) {
        const int w = (int)std::min<int64_t>(SB, b - k0);
        double* Akk = A + k0 * ld + k0;
        hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(256), 0, s, ld, k0, w, A);
        // row panel: rows k (w of them), all columns outside the block
        hipLaunchKernelGGL(k_gemm, dim3(tn, 1), dim3(256), 0, s, (int64_t)w, (int64_t)b, w, 1.0, (const double*)Akk,
                           ld, (const double*)(A + k0 * ld), ld, 0.0, A + k0 * ld, ld, (int64_t)0, (int64_t)0, k0,
                           k0 + w);
        // trailing update on all rows/columns outside the block
        hipLaunchKernelGGL(k_gemm, dim3(tn, tn), dim3(256), 0, s, (int64_t)b, (int64_t)b, w, -1.0,
                           (const double*)(A + k0), ld, (const double*)(A + k0 * ld), ld, 1.0, A, ld, k0, k0 + w, k0,
                           k0 + w);
        // column panel: all rows outside the block, columns k
        hipLaunchKernelGGL(k_gemm, dim3(1, tn), dim3(256), 0, s, (int64_t)b, (int64_t)w, w, -1.0,
                           (const double*)(A + k0), ld, (const double*)Akk, ld, 0.0, A + k0, ld, k0, k0 + w,
                           (int64_t)0, (int64_t)0);
    }
}

}  // namespace

size_t dense_invert_tmp_doubles(int64_t n) {
    const int64_t b = std::min<int64_t>(DB, std::max<int64_t>(n, 1));
    return (size_t)(2 * n * b + b * b);
}

fem_status dense_invert(int64_t n, double* A, double* tmp, hipStream_t s) {
    if (n <= 0) return FEM_OK;
    if (!A || !tmp) {
        set_error("dense inversion: NULL matrix or scratch");
        return FEM_ERR_INVALID_ARG;
    }
    const int64_t bmax = std::min<int64_t>(DB, n);
    double* W = tmp;
    double* Vs = W + n * bmax;
    double* Pb = Vs + n * bmax;
    const int64_t nt = (n + UT - 1) / UT;
    const unsigned ntiles = (unsigned)(nt * (nt + 1) / 2);
    const unsigned rt = (unsigned)((n + SB - 1) / SB);
    for (int64_t k0 = 0; k0 < n; k0 += DB) {
        const int b = (int)std::min<int64_t>(DB, n - k0);
        const unsigned ct = (unsigned)((b + SB - 1) / SB);
        hipLaunchKernelGGL(k_gj_gather, dim3(rt, ct), dim3(256), 0, s, n, b, k0, (const double*)A, W);
        hipLaunchKernelGGL(k_gj_block, dim3((unsigned)((b * b + 255) / 256)), dim3(256), 0, s, n, b, k0,
                           (const double*)A, Pb);
        invert_block(b, b, Pb, s);
        // Vs = s (W P): rows above K negated, rows below as they are
        if (k0 > 0)
            hipLaunchKernelGGL(k_gemm, dim3(ct, (unsigned)((k0 + GT - 1) / GT)), dim3(256), 0, s, k0, (int64_t)b, b,
                               -1.0, (const double*)W, (int64_t)b, (const double*)Pb, (int64_t)b, 0.0, Vs, (int64_t)b,
                               (int64_t)0, (int64_t)0, (int64_t)0, (int64_t)0);
        const int64_t below = n - k0 - b;
        if (below > 0)
            hipLaunchKernelGGL(k_gemm, dim3(ct, (unsigned)((below + GT - 1) / GT)), dim3(256), 0, s, below,
                               (int64_t)b, b, 1.0, (const double*)(W + (k0 + b) * b), (int64_t)b, (const double*)Pb,
                               (int64_t)b, 0.0, Vs + (k0 + b) * b, (int64_t)b, (int64_t)0, (int64_t)0, (int64_t)0,
                               (int64_t)0);
        if (n > b)
            hipLaunchKernelGGL(k_gj_update, dim3(ntiles), dim3(256), 0, s, n, b, k0, (const double*)W,
                               (const double*)Vs, A);
        hipLaunchKernelGGL(k_gj_panels, dim3(rt, ct), dim3(256), 0, s, n, b, k0, (const double*)Vs,
                           (const double*)Pb, A);
    }
    return check_launch("dense inversion");
}

}  // namespace fem
