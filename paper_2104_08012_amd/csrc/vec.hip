// Vector kernels of the multigrid-CG solver: deterministic dot products, axpy forms, the fused
// Chebyshev update, precision casts, coefficient injection, and the dense coarse-grid kernels
// (probing assembly, packed symmetric tiles and their matrix-vector product; the inversion is in
// dense.hip).
#include "vec.hpp"

namespace fem {

namespace {
constexpr int VT = 256;

inline unsigned grid_for(int64_t n, int per_thread = 1) {
    int64_t g = (n + (int64_t)VT * per_thread - 1) / ((int64_t)VT * per_thread);
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 0x7fffffff));
}

// ---------------- deterministic dot products ----------------
// Stage 1: block b sums the elements i = b*chunk .. (b+1)*chunk-1 with a fixed per-thread stride
// and a fixed LDS tree; stage 2: one block sums the partials in a fixed tree.  The result does
// not depend on timing, only on n and the fixed grid.
constexpr int DOT_BLOCKS = 1024;

template <typename T, int NPAIR>
__global__ void __launch_bounds__(VT) k_dot_partial(int64_t n, DotPairs<T> pr, double* partial) {
    __shared__ double sh[NPAIR][VT];
    const int64_t chunk = (n + DOT_BLOCKS - 1) / DOT_BLOCKS;
    const int64_t lo = blockIdx.x * chunk, hi = (lo + chunk < n) ? lo + chunk : n;
    double acc[NPAIR];
#pragma unroll
    for (int p = 0; p < NPAIR; ++p) acc[p] = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += VT) {
#pragma unroll
        for (int p = 0; p < NPAIR; ++p) acc[p] += (double)pr.x[p][i] * (double)pr.y[p][i];
    }
#pragma unroll
    for (int p = 0; p < NPAIR; ++p) sh[p][threadIdx.x] = acc[p];
    __syncthreads();
    for (int s = VT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
#pragma unroll
            for (int p = 0; p < NPAIR; ++p) sh[p][threadIdx.x] += sh[p][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < NPAIR) partial[threadIdx.x * DOT_BLOCKS + blockIdx.x] = sh[threadIdx.x][0];
}

// the partials' fixed tree, leaving the sums in sh[p][0]
template <int NPAIR>
__device__ __forceinline__ void dot_final_tree(const double* partial, double (*sh)[VT]) {
#pragma unroll
    for (int p = 0; p < NPAIR; ++p) {
        double a = 0.0;
        for (int i = threadIdx.x; i < DOT_BLOCKS; i += VT) a += partial[p * DOT_BLOCKS + i];
        sh[p][threadIdx.x] = a;
    }
    __syncthreads();
    for (int s = VT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
#pragma unroll
            for (int p = 0; p < NPAIR; ++p) sh[p][threadIdx.x] += sh[p][threadIdx.x + s];
        __syncthreads();
    }
}

template <int NPAIR>
__global__ void __launch_bounds__(VT) k_dot_final(const double* partial, double* out) {
    __shared__ double sh[NPAIR][VT];
    dot_final_tree<NPAIR>(partial, sh);
    if (threadIdx.x < NPAIR) out[threadIdx.x] = sh[threadIdx.x][0];
}

// ---------------- elementwise ----------------
template <typename T>
__global__ void k_axpby(int64_t n, double a, const T* __restrict__ x, double b, T* y) {
    const int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x;
    if (i < n) y[i] = (T)(b == 0.0 ? a * (double)x[i] : a * (double)x[i] + b * (double)y[i]);   // b = 0: y not read
}

// Device-resident CG scalars (indices into the solver's scalar block, see vec.hpp).
// alpha = rz / pq, or 0 with flag bit 1 when p^T A p is not positive and finite.
__device__ __forceinline__ void cg_alpha(double* sc) {
    const double pq = sc[CG_PQ], rz = sc[CG_RZ];
    const bool ok = pq > 0.0 && pq < INFINITY;
    sc[CG_ALPHA] = ok ? rz / pq : 0.0;
    if (!ok) sc[CG_FLAG] = (double)((int)sc[CG_FLAG] | 1);
}

// beta (Fletcher-Reeves rz_new / rz, or Polak-Ribiere -alpha qz / rz) and rz = rz_new; beta = 0
// with flag bit 2 when r^T z is not positive and finite.
__device__ __forceinline__ void cg_beta(double* sc, int flexible) {
    const double rzn = sc[CG_RZNEW], rz = sc[CG_RZ];
    const bool ok = rzn > 0.0 && rzn < INFINITY;
    sc[CG_BETA] = !ok ? 0.0 : flexible ? -sc[CG_ALPHA] * sc[CG_QZ] / rz : rzn / rz;
    sc[CG_RZ] = rzn;
    if (!ok) sc[CG_FLAG] = (double)((int)sc[CG_FLAG] | 2);
}

// The last reduction stage of p^T q fused with alpha (one launch instead of two; the same tree).
__global__ void __launch_bounds__(VT) k_dot_final_alpha(const double* partial, double* sc) {
    __shared__ double sh[1][VT];
    dot_final_tree<1>(partial, sh);
    if (threadIdx.x == 0) {
        sc[CG_PQ] = sh[0][0];
        cg_alpha(sc);
    }
}

// The last reduction stage of (r^T z, q^T z) fused with beta.
__global__ void __launch_bounds__(VT) k_dot_final_beta(const double* partial, double* sc, int flexible) {
    __shared__ double sh[2][VT];
    dot_final_tree<2>(partial, sh);
    if (threadIdx.x == 0) {
        sc[CG_RZNEW] = sh[0][0];
        sc[CG_QZ] = sh[1][0];
        cg_beta(sc, flexible);
    }
}

// x += alpha p ; r -= alpha q, with the first reduction stage of r^T r over the updated r in
// the same pass (the chunks, strides and tree of k_dot_partial, so r^T r is bitwise the one a
// separate dot product would give).
__global__ void __launch_bounds__(VT) k_cg_update_dot(int64_t n, const double* __restrict__ sc, const double* __restrict__ p,
                                                    const double* __restrict__ q, double* __restrict__ x,
                                                    double* __restrict__ r, double* __restrict__ partial) {
    __shared__ double sh[VT];
    const double alpha = sc[CG_ALPHA];
    const int64_t chunk = (n + DOT_BLOCKS - 1) / DOT_BLOCKS;
    const int64_t lo = blockIdx.x * chunk, hi = (lo + chunk < n) ? lo + chunk : n;
    double acc = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += VT) {
        x[i] += alpha * p[i];
        const double rn = r[i] - alpha * q[i];
        r[i] = rn;
        acc += rn * rn;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = VT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

// x += alpha p ; r -= alpha q with alpha read from device memory
__global__ void k_cg_update_dev(int64_t n, const double* __restrict__ sc, const double* __restrict__ p,
                                const double* __restrict__ q, double* __restrict__ x, double* __restrict__ r) {
    const int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x;
    if (i < n) {
        const double alpha = sc[CG_ALPHA];
        x[i] += alpha * p[i];
        r[i] -= alpha * q[i];
    }
}

// p = z + beta p with beta read from device memory
__global__ void k_cg_direction_dev(int64_t n, const double* __restrict__ sc, const double* __restrict__ z,
                                   double* __restrict__ p) {
    const int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x;
    if (i < n) p[i] = z[i] + sc[CG_BETA] * p[i];
}

// Chebyshev step: d = c1 d + c2 dinv r ; x = (init ? d : x + d)   (dinv NULL: r is already
// preconditioned)
template <typename T>
__global__ void k_cheb(int64_t n, T c1, T c2, const T* __restrict__ dinv, const T* __restrict__ r,
                       T* __restrict__ d, T* __restrict__ x, int init) {
    const int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x;
    if (i < n) {
        const T dn = c1 * d[i] + (dinv ? c2 * dinv[i] * r[i] : c2 * r[i]);
        d[i] = dn;
        x[i] = init ? dn : x[i] + dn;
    }
}

// first Chebyshev step: d = c2 dinv r ; x = (init ? d : x + d)
template <typename T>
__global__ void k_cheb0(int64_t n, T c2, const T* __restrict__ dinv, const T* __restrict__ r,
                        T* __restrict__ d, T* __restrict__ x, int init) {
    const int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x;
    if (i < n) {
        const T dn = dinv ? c2 * dinv[i] * r[i] : c2 * r[i];
        d[i] = dn;
        x[i] = init ? dn : x[i] + dn;
    }
}

template <typename A, typename B>
__global__ void k_cast(int64_t n, const A* __restrict__ x, B* __restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x;
    if (i < n) y[i] = (B)x[i];
}

template <typename T>
__global__ void k_fill(int64_t n, T v, T* __restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x;
    if (i < n) y[i] = v;
}

// y = 1 / x (Jacobi scaling from the diagonal)
template <typename T>
__global__ void k_recip(int64_t n, const T* __restrict__ x, T* __restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x;
    if (i < n) y[i] = T(1) / x[i];
}

// y = x * s  (elementwise product)
template <typename T>
__global__ void k_mul(int64_t n, const T* __restrict__ x, const T* __restrict__ s, T* __restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x;
    if (i < n) y[i] = x[i] * s[i];
}

template <typename T>
__global__ void k_div(int64_t n, const T* __restrict__ x, const T* __restrict__ s, T* __restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x;
    if (i < n) y[i] = x[i] / s[i];
}

// k on the vertex lattice of a coarser level by injection: k_c(i,j,k) = k_f(2^s i, 2^s j, 2^s k)
template <typename T>
__global__ void k_inject(int nc, int stride, int nf, const double* __restrict__ kf, T* __restrict__ kc) {
    const int64_t t = (int64_t)blockIdx.x * VT + threadIdx.x;
    const int64_t n1 = nc + 1;
    if (t >= n1 * n1 * n1) return;
    const int i = (int)(t % n1), j = (int)((t / n1) % n1), k = (int)(t / (n1 * n1));
    const int64_t f1 = nf + 1;
    kc[t] = (T)kf[(int64_t)i * stride + f1 * ((int64_t)j * stride + f1 * (int64_t)k * stride)];
}

// Random start vector from a counter-based generator (SplitMix64 of the index), in [-1, 1),
// zero on boundary dofs of the (L^3) lattice.
__global__ void k_random(int64_t n, int L, uint64_t seed, double* __restrict__ v) {
    const int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x;
    if (i >= n) return;
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(i + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);
    const int I = (int)(i % L), J = (int)((i / L) % L), K = (int)(i / ((int64_t)L * L));
    const bool bnd = I == 0 || J == 0 || K == 0 || I == L - 1 || J == L - 1 || K == L - 1;
    v[i] = bnd ? 0.0 : 2.0 * u - 1.0;
}

// ---------------- dense coarse solve ----------------
// Probing vector for colour (c0, c1, c2) of period S: ones at interior lattice points congruent
// to the colour, zero elsewhere.
__global__ void k_probe_fill(int L, int S, int c0, int c1, int c2, double* __restrict__ v) {
    const int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x;
    const int64_t N = (int64_t)L * L * L;
    if (i >= N) return;
    const int I = (int)(i % L), J = (int)((i / L) % L), K = (int)(i / ((int64_t)L * L));
    const bool interior = I > 0 && J > 0 && K > 0 && I < L - 1 && J < L - 1 && K < L - 1;
    v[i] = (interior && I % S == c0 && J % S == c1 && K % S == c2) ? 1.0 : 0.0;
}

// For every interior row i, the column j of the colour with |i - j|_inf <= p is unique (S = 2p+1)
// and A_ij = (A v)_i.  Writes A_dense[row][col] over interior indices.
__global__ void k_probe_extract(int L, int p, int S, int c0, int c1, int c2, const double* __restrict__ y,
                                double* __restrict__ A) {
    const int M = L - 2;
    const int64_t t = (int64_t)blockIdx.x * VT + threadIdx.x;
    if (t >= (int64_t)M * M * M) return;
    const int I = (int)(t % M) + 1, J = (int)((t / M) % M) + 1, K = (int)(t / ((int64_t)M * M)) + 1;
    const int c[3] = {c0, c1, c2};
    const int X[3] = {I, J, K};
    int Y[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        int lo = X[d] - p;
        int r = ((c[d] - lo) % S + S) % S;
        Y[d] = lo + r;
    }
    if (Y[0] < 1 || Y[1] < 1 || Y[2] < 1 || Y[0] > L - 2 || Y[1] > L - 2 || Y[2] > L - 2) return;
    const int64_t col = (Y[0] - 1) + (int64_t)M * ((Y[1] - 1) + (int64_t)M * (Y[2] - 1));
    const int64_t g = I + (int64_t)L * (J + (int64_t)L * K);
    A[t * (int64_t)M * M * M + col] = y[g];
}

// Symmetric coarse inverse in packed lower tiles: tile (I, J), I >= J, of 64 x 64 entries
// (row-major inside the tile, zero beyond n) at offset (I (I + 1) / 2 + J) * 4096.
constexpr int ST = 64;

__device__ __forceinline__ void tile_of(int64_t t, int& I, int& J) {
    int i = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((int64_t)(i + 1) * (i + 2) / 2 <= t) ++i;
    while ((int64_t)i * (i + 1) / 2 > t) --i;
    I = i;
    J = (int)(t - (int64_t)i * (i + 1) / 2);
}

// Ap tile (I, J) = A_IJ from the lower triangle the inversion keeps, diagonal tiles
// (A_II + A_II^T) / 2, stored in TO (FP64, or FP32 for the mixed-precision preconditioner: rounded
// once from the FP64 inverse).
template <typename TO>
__global__ void __launch_bounds__(256) k_sym_pack(int64_t n, const double* __restrict__ A, TO* __restrict__ Ap) {
    int I, J;
    tile_of(blockIdx.x, I, J);
    TO* out = Ap + (int64_t)blockIdx.x * ST * ST;
    for (int e = threadIdx.x; e < ST * ST; e += 256) {
        const int64_t i = (int64_t)I * ST + e / ST, j = (int64_t)J * ST + e % ST;
        double v = 0.0;
        if (i < n && j < n) v = I == J ? 0.5 * (A[i * n + j] + A[j * n + i]) : A[i * n + j];
        out[e] = (TO)v;
    }
}

// 16-byte vector of tile entries
template <typename TA>
struct Vec16;
template <>
struct Vec16<double> {
    using type = double2;
    static constexpr int n = 2;
    __device__ static double get(const double2& v, int k) { return k == 0 ? v.x : v.y; }
};
template <>
struct Vec16<float> {
    using type = float4;
    static constexpr int n = 4;
    __device__ static float get(const float4& v, int k) { return k == 0 ? v.x : k == 1 ? v.y : k == 2 ? v.z : v.w; }
};

// Per tile t = (I, J): prow[t] = A_IJ x_J and, off the diagonal, pcol[t] = A_IJ^T x_I
// (64 entries each), accumulated in FP64 whatever the tile's storage type TA.  Persistent blocks:
// block b takes tiles b, b + gridDim.x, ...; the next two tiles are loaded into registers (16-byte
// loads) while the current one, staged in LDS, is multiplied, so the stream of tile reads does not
// stop for the arithmetic.  Thread (e, q) of the 256 sums a quarter (16 terms, fixed order) of row
// e and of column e, and the quarters are added in order q = 0..3.
template <typename TA, int DEPTH>
__global__ void __launch_bounds__(256) k_sym_tiles(int64_t n, int64_t ntiles, const TA* __restrict__ Ap,
                                                   const double* __restrict__ xc, double* __restrict__ prow,
                                                   double* __restrict__ pcol) {
    using V = Vec16<TA>;
    using VT16 = typename V::type;
    constexpr int NPT = ST * ST / V::n / 256;   // vectors per thread and tile
    __shared__ TA sa[ST][ST + 1];
    __shared__ double sx[2][ST];
    __shared__ double sq[2][4][ST];
    const int64_t G = gridDim.x;
    int64_t t = blockIdx.x;
    if (t >= ntiles) return;
    VT16 cur[NPT], nxt[NPT];
    {
        const VT16* tile = reinterpret_cast<const VT16*>(Ap + t * ST * ST);
#pragma unroll
        for (int k = 0; k < NPT; ++k) cur[k] = tile[threadIdx.x + 256 * k];
        if (DEPTH == 2 && t + G < ntiles) {
            const VT16* tn = reinterpret_cast<const VT16*>(Ap + (t + G) * ST * ST);
#pragma unroll
            for (int k = 0; k < NPT; ++k) nxt[k] = tn[threadIdx.x + 256 * k];
        }
    }
    const int e = threadIdx.x % ST, q = threadIdx.x / ST;
    for (; t < ntiles; t += G) {
        int I, J;
        tile_of(t, I, J);
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int pe = threadIdx.x + 256 * k, r = (V::n * pe) / ST, c = (V::n * pe) % ST;
#pragma unroll
            for (int u = 0; u < V::n; ++u) sa[r][c + u] = V::get(cur[k], u);
        }
        if (threadIdx.x < ST) {
            const int64_t jj = (int64_t)J * ST + threadIdx.x, ii = (int64_t)I * ST + threadIdx.x;
            sx[0][threadIdx.x] = jj < n ? xc[jj] : 0.0;
            sx[1][threadIdx.x] = ii < n ? xc[ii] : 0.0;
        }
        __syncthreads();
        if constexpr (DEPTH == 2) {
#pragma unroll
            for (int k = 0; k < NPT; ++k) cur[k] = nxt[k];
            const int64_t t2 = t + 2 * G;
            if (t2 < ntiles) {
                const VT16* tile = reinterpret_cast<const VT16*>(Ap + t2 * ST * ST);
#pragma unroll
                for (int k = 0; k < NPT; ++k) nxt[k] = tile[threadIdx.x + 256 * k];
            }
        } else if (t + G < ntiles) {
            const VT16* tile = reinterpret_cast<const VT16*>(Ap + (t + G) * ST * ST);
#pragma unroll
            for (int k = 0; k < NPT; ++k) cur[k] = tile[threadIdx.x + 256 * k];
        }
        double ar = 0.0, ac = 0.0;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int c = q * 16 + k;
            ar += (double)sa[e][c] * sx[0][c];
            ac += (double)sa[c][e] * sx[1][c];
        }
        sq[0][q][e] = ar;
        sq[1][q][e] = ac;
        __syncthreads();
        if (q == 0) {
            prow[t * ST + e] = ((sq[0][0][e] + sq[0][1][e]) + sq[0][2][e]) + sq[0][3][e];
        } else if (q == 1 && I != J) {
            pcol[t * ST + e] = ((sq[1][0][e] + sq[1][1][e]) + sq[1][2][e]) + sq[1][3][e];
        }
        __syncthreads();
    }
}

// y at the interior lattice points of row block I: the terms A_IJ x_J, from prow (J <= I) or
// pcol of tile (J, I) (J > I), summed by four groups of 64 threads over J = g, g + 4, ... and the
// four group sums added in group order (a fixed order).
__global__ void __launch_bounds__(4 * ST) k_sym_reduce(int L, int64_t n, int nt, const double* __restrict__ prow,
                                                       const double* __restrict__ pcol, double* __restrict__ yl) {
    __shared__ double sg[4][ST];
    const int I = blockIdx.x, r = threadIdx.x % ST, g = threadIdx.x / ST;
    double acc = 0.0;
#pragma unroll 4
    for (int J = g; J < nt; J += 4) {
        const double* src = J <= I ? prow + ((int64_t)I * (I + 1) / 2 + J) * ST : pcol + ((int64_t)J * (J + 1) / 2 + I) * ST;
        acc += src[r];
    }
    sg[g][r] = acc;
    __syncthreads();
    if (g != 0) return;
    acc = ((sg[0][r] + sg[1][r]) + sg[2][r]) + sg[3][r];
    const int64_t row = (int64_t)I * ST + r;
    if (row >= n) return;
    const int M = L - 2;
    const int i = (int)(row % M) + 1, j = (int)((row / M) % M) + 1, k = (int)(row / ((int64_t)M * M)) + 1;
    yl[i + (int64_t)L * (j + (int64_t)L * k)] = acc;
}

// gather interior entries of a lattice vector into a compact vector
__global__ void k_gather_interior(int L, const double* __restrict__ xl, double* __restrict__ xc) {
    const int M = L - 2;
    const int64_t t = (int64_t)blockIdx.x * VT + threadIdx.x;
    if (t >= (int64_t)M * M * M) return;
    const int I = (int)(t % M) + 1, J = (int)((t / M) % M) + 1, K = (int)(t / ((int64_t)M * M)) + 1;
    xc[t] = xl[I + (int64_t)L * (J + (int64_t)L * K)];
}

template <typename T>
__global__ void k_zero_boundary(int L, T* __restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x;
    const int64_t N = (int64_t)L * L * L;
    if (i >= N) return;
    const int I = (int)(i % L), J = (int)((i / L) % L), K = (int)(i / ((int64_t)L * L));
    if (I == 0 || J == 0 || K == 0 || I == L - 1 || J == L - 1 || K == L - 1) y[i] = T(0);
}

}  // namespace

// ---------------- launchers ----------------
template <typename T>
void dot_launch(int npair, int64_t n, const DotPairs<T>& pr, double* partial, double* out, hipStream_t s) {
    if (npair == 1) {
        hipLaunchKernelGGL((k_dot_partial<T, 1>), dim3(DOT_BLOCKS), dim3(VT), 0, s, n, pr, partial);
        hipLaunchKernelGGL((k_dot_final<1>), dim3(1), dim3(VT), 0, s, partial, out);
    } else if (npair == 2) {
        hipLaunchKernelGGL((k_dot_partial<T, 2>), dim3(DOT_BLOCKS), dim3(VT), 0, s, n, pr, partial);
        hipLaunchKernelGGL((k_dot_final<2>), dim3(1), dim3(VT), 0, s, partial, out);
    } else {
        hipLaunchKernelGGL((k_dot_partial<T, 3>), dim3(DOT_BLOCKS), dim3(VT), 0, s, n, pr, partial);
        hipLaunchKernelGGL((k_dot_final<3>), dim3(1), dim3(VT), 0, s, partial, out);
    }
}
template void dot_launch<double>(int, int64_t, const DotPairs<double>&, double*, double*, hipStream_t);
template void dot_launch<float>(int, int64_t, const DotPairs<float>&, double*, double*, hipStream_t);
size_t dot_partial_doubles() { return 3 * DOT_BLOCKS; }

template <typename T>
void axpby_launch(int64_t n, double a, const T* x, double b, T* y, hipStream_t s) {
    hipLaunchKernelGGL((k_axpby<T>), dim3(grid_for(n)), dim3(VT), 0, s, n, a, x, b, y);
}
template void axpby_launch<double>(int64_t, double, const double*, double, double*, hipStream_t);
template void axpby_launch<float>(int64_t, double, const float*, double, float*, hipStream_t);

void dot_alpha_launch(int64_t n, const double* p, const double* q, double* partial, double* sc, hipStream_t s) {
    DotPairs<double> pr{{p, nullptr, nullptr}, {q, nullptr, nullptr}};
    hipLaunchKernelGGL((k_dot_partial<double, 1>), dim3(DOT_BLOCKS), dim3(VT), 0, s, n, pr, partial);
    hipLaunchKernelGGL(k_dot_final_alpha, dim3(1), dim3(VT), 0, s, partial, sc);
}
void dot_beta_launch(int64_t n, const double* r, const double* z, const double* q, double* partial, double* sc,
                     bool flexible, hipStream_t s) {
    DotPairs<double> pr{{r, q, nullptr}, {z, z, nullptr}};
    hipLaunchKernelGGL((k_dot_partial<double, 2>), dim3(DOT_BLOCKS), dim3(VT), 0, s, n, pr, partial);
    hipLaunchKernelGGL(k_dot_final_beta, dim3(1), dim3(VT), 0, s, partial, sc, flexible ? 1 : 0);
}
void cg_update_dot_launch(int64_t n, const double* sc, const double* p, const double* q, double* x, double* r,
                          double* partial, double* rr, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_update_dot, dim3(DOT_BLOCKS), dim3(VT), 0, s, n, sc, p, q, x, r, partial);
    hipLaunchKernelGGL((k_dot_final<1>), dim3(1), dim3(VT), 0, s, partial, rr);
}
void cg_update_dev_launch(int64_t n, const double* sc, const double* p, const double* q, double* x, double* r,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_cg_update_dev, dim3(grid_for(n)), dim3(VT), 0, s, n, sc, p, q, x, r);
}
void cg_direction_dev_launch(int64_t n, const double* sc, const double* z, double* p, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_direction_dev, dim3(grid_for(n)), dim3(VT), 0, s, n, sc, z, p);
}

template <typename T>
void cheb_launch(int64_t n, double c1, double c2, const T* dinv, const T* r, T* d, T* x, bool first, bool init,
                 hipStream_t s) {
    if (first)
        hipLaunchKernelGGL((k_cheb0<T>), dim3(grid_for(n)), dim3(VT), 0, s, n, (T)c2, dinv, r, d, x, init ? 1 : 0);
    else
        hipLaunchKernelGGL((k_cheb<T>), dim3(grid_for(n)), dim3(VT), 0, s, n, (T)c1, (T)c2, dinv, r, d, x, init ? 1 : 0);
}
template void cheb_launch<double>(int64_t, double, double, const double*, const double*, double*, double*, bool, bool, hipStream_t);
template void cheb_launch<float>(int64_t, double, double, const float*, const float*, float*, float*, bool, bool, hipStream_t);

template <typename A, typename B>
void cast_launch(int64_t n, const A* x, B* y, hipStream_t s) {
    hipLaunchKernelGGL((k_cast<A, B>), dim3(grid_for(n)), dim3(VT), 0, s, n, x, y);
}
template void cast_launch<double, float>(int64_t, const double*, float*, hipStream_t);
template void cast_launch<float, double>(int64_t, const float*, double*, hipStream_t);
template void cast_launch<double, double>(int64_t, const double*, double*, hipStream_t);
template void cast_launch<float, float>(int64_t, const float*, float*, hipStream_t);

template <typename T>
void fill_launch(int64_t n, T v, T* y, hipStream_t s) {
    hipLaunchKernelGGL((k_fill<T>), dim3(grid_for(n)), dim3(VT), 0, s, n, v, y);
}
template void fill_launch<double>(int64_t, double, double*, hipStream_t);
template void fill_launch<float>(int64_t, float, float*, hipStream_t);

template <typename T>
void recip_launch(int64_t n, const T* x, T* y, hipStream_t s) {
    hipLaunchKernelGGL((k_recip<T>), dim3(grid_for(n)), dim3(VT), 0, s, n, x, y);
}
template void recip_launch<double>(int64_t, const double*, double*, hipStream_t);
template void recip_launch<float>(int64_t, const float*, float*, hipStream_t);

template <typename T>
void mul_launch(int64_t n, const T* x, const T* sc, T* y, hipStream_t s) {
    hipLaunchKernelGGL((k_mul<T>), dim3(grid_for(n)), dim3(VT), 0, s, n, x, sc, y);
}
template void mul_launch<double>(int64_t, const double*, const double*, double*, hipStream_t);

template <typename T>
void div_launch(int64_t n, const T* x, const T* sc, T* y, hipStream_t s) {
    hipLaunchKernelGGL((k_div<T>), dim3(grid_for(n)), dim3(VT), 0, s, n, x, sc, y);
}
template void div_launch<double>(int64_t, const double*, const double*, double*, hipStream_t);

template <typename T>
void inject_launch(int nc, int stride, int nf, const double* kf, T* kc, hipStream_t s) {
    const int64_t n1 = nc + 1;
    hipLaunchKernelGGL((k_inject<T>), dim3(grid_for(n1 * n1 * n1)), dim3(VT), 0, s, nc, stride, nf, kf, kc);
}
template void inject_launch<double>(int, int, int, const double*, double*, hipStream_t);
template void inject_launch<float>(int, int, int, const double*, float*, hipStream_t);

void random_launch(int64_t n, int L, uint64_t seed, double* v, hipStream_t s) {
    hipLaunchKernelGGL(k_random, dim3(grid_for(n)), dim3(VT), 0, s, n, L, seed, v);
}

void probe_fill_launch(int L, int S, int c0, int c1, int c2, double* v, hipStream_t s) {
    const int64_t N = (int64_t)L * L * L;
    hipLaunchKernelGGL(k_probe_fill, dim3(grid_for(N)), dim3(VT), 0, s, L, S, c0, c1, c2, v);
}
void probe_extract_launch(int L, int p, int S, int c0, int c1, int c2, const double* y, double* A, hipStream_t s) {
    const int64_t M = L - 2;
    hipLaunchKernelGGL(k_probe_extract, dim3(grid_for(M * M * M)), dim3(VT), 0, s, L, p, S, c0, c1, c2, y, A);
}

int64_t sym_tiles(int64_t n) {
    const int64_t nt = (n + ST - 1) / ST;
    return nt * (nt + 1) / 2;
}
size_t sym_packed_doubles(int64_t n) { return (size_t)sym_tiles(n) * ST * ST; }
size_t sym_partial_doubles(int64_t n) { return (size_t)2 * sym_tiles(n) * ST; }

template <typename TA>
void sym_pack_launch(int64_t n, const double* A, TA* Ap, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL((k_sym_pack<TA>), dim3((unsigned)sym_tiles(n)), dim3(256), 0, s, n, A, Ap);
}
template void sym_pack_launch<double>(int64_t, const double*, double*, hipStream_t);
template void sym_pack_launch<float>(int64_t, const double*, float*, hipStream_t);

#ifndef FEM_TILE_DEPTH64
#define FEM_TILE_DEPTH64 1
#endif
#ifndef FEM_TILE_DEPTH32
#define FEM_TILE_DEPTH32 2
#endif
// tiles loaded ahead per block: the FP64 instance keeps 4 blocks per CU with one, the FP32 one
// (16-byte loads of four entries) gains from two
template <typename TA>
constexpr int kTileDepth = sizeof(TA) == 8 ? FEM_TILE_DEPTH64 : FEM_TILE_DEPTH32;

template <typename TA>
void sym_solve_launch(int L, const TA* Ap, const double* xl, double* xc, double* part, double* yl,
                      hipStream_t s) {
    const int64_t M = L - 2, m = M * M * M, ntl = sym_tiles(m);
    const int nt = (int)((m + ST - 1) / ST);
    const int64_t N = (int64_t)L * L * L;
    hipLaunchKernelGGL((k_zero_boundary<double>), dim3(grid_for(N)), dim3(VT), 0, s, L, yl);
    if (m == 0) return;   // every dof on the boundary
    hipLaunchKernelGGL(k_gather_interior, dim3(grid_for(m)), dim3(VT), 0, s, L, xl, xc);
    double* prow = part;
    double* pcol = part + ntl * ST;
    // persistent blocks: as many as are resident at once (occupancy of this instance times the
    // CU count, queried once per tile type)
    static int resident = 0;
    if (resident == 0) {
        int dev = 0, cus = 0, per = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_sym_tiles<TA, kTileDepth<TA>>, 256, 0) == hipSuccess && cus > 0 &&
            per > 0)
            resident = cus * per;
        else
            resident = 256;
    }
    const int64_t nblk = std::min<int64_t>(ntl, resident);
    hipLaunchKernelGGL((k_sym_tiles<TA, kTileDepth<TA>>), dim3((unsigned)nblk), dim3(256), 0, s, m, ntl, Ap, (const double*)xc,
                       prow, pcol);
    hipLaunchKernelGGL(k_sym_reduce, dim3((unsigned)nt), dim3(4 * ST), 0, s, L, m, nt, (const double*)prow,
                       (const double*)pcol, yl);
}
template void sym_solve_launch<double>(int, const double*, const double*, double*, double*, double*, hipStream_t);
template void sym_solve_launch<float>(int, const float*, const double*, double*, double*, double*, hipStream_t);


}  // namespace fem
