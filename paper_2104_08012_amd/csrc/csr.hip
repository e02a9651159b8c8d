// Assembled operator (the representation the paper's solvers use, §4: sparse matrices and SpMV):
// element matrices on the GPU, a deterministic per-entry sum into CSR values, and SpMV.
//
//  * k_elem: one thread per cell, A_K[i][j] = sum_q w_q k(x_q) (D_q^T G D_q)[i][j] with the
//    runtime quadrature tabulation of the stiffness kernels (same rule as the matrix-free
//    action), written entry-major E[(i nloc + j) C + c] so that neighbouring cells store
//    contiguously.
//  * k_csr_gather: one thread per stored entry, the sum of its element-matrix contributions in
//    the fixed (ascending cell) order the host listed, or the identity row / zero column of a
//    Dirichlet dof (symmetric elimination, as in the matrix-free operator).
//  * k_spmv: y = A x with LANES lanes per row (each lane's entries in ascending order, their loads
//    issued four at a time) and a fixed-shape shuffle reduction, so results are bitwise
//    reproducible.
#include "csr.hpp"

namespace fem {

namespace {

constexpr int VT = 256;

template <int NL>
__global__ void __launch_bounds__(VT) k_elem(int64_t C, int n, int p, int L, const int32_t* __restrict__ map,
                                            const double* __restrict__ G, const double* __restrict__ tab, int nq,
                                            const double* __restrict__ k, double* __restrict__ E) {
    constexpr int stride = 1 + 4 + 3 * NL;
    const int64_t c = (int64_t)blockIdx.x * VT + threadIdx.x;
    if (c >= C) return;
    const double g00 = G[c], g11 = G[C + c], g22 = G[2 * C + c], g01 = G[3 * C + c], g02 = G[4 * C + c],
                 g12 = G[5 * C + c];
    double kv[4] = {1.0, 1.0, 1.0, 1.0};
    if (k) {
        // vertex v of the cell is local node v; its lattice point (I, J, K) / p is the vertex
        const int n1 = n + 1;
        for (int v = 0; v < 4; ++v) {
            const int32_t gd = map[(int64_t)v * C + c] & 0x7fffffff;
            const int I = gd % L, J = (gd / L) % L, K = gd / (L * L);
            kv[v] = k[(I / p) + n1 * ((J / p) + n1 * (K / p))];
        }
    }
    for (int i = 0; i < NL; ++i) {
        double acc[NL];
#pragma unroll
        for (int j = 0; j < NL; ++j) acc[j] = 0.0;
        for (int q = 0; q < nq; ++q) {
            const double* t = tab + (size_t)q * stride;
            double s = t[0];
            if (k) s *= t[1] * kv[0] + t[2] * kv[1] + t[3] * kv[2] + t[4] * kv[3];
            const double* D = t + 5;
            const double di0 = D[i], di1 = D[NL + i], di2 = D[2 * NL + i];
            const double u0 = s * (g00 * di0 + g01 * di1 + g02 * di2);
            const double u1 = s * (g01 * di0 + g11 * di1 + g12 * di2);
            const double u2 = s * (g02 * di0 + g12 * di1 + g22 * di2);
#pragma unroll
            for (int j = 0; j < NL; ++j) acc[j] += u0 * D[j] + u1 * D[NL + j] + u2 * D[2 * NL + j];
        }
#pragma unroll
        for (int j = 0; j < NL; ++j) E[(int64_t)(i * NL + j) * C + c] = acc[j];
    }
}

template <typename T>
__global__ void __launch_bounds__(VT) k_csr_gather(int64_t nnz, const int64_t* __restrict__ cptr,
                                                  const int32_t* __restrict__ cidx, const uint8_t* __restrict__ flag,
                                                  const double* __restrict__ E, T* __restrict__ val) {
    const int64_t e = (int64_t)blockIdx.x * VT + threadIdx.x;
    if (e >= nnz) return;
    const uint8_t f = flag[e];
    double v = 0.0;
    if (f == CSR_SUM) {
        for (int64_t t = cptr[e]; t < cptr[e + 1]; ++t) v += E[(uint32_t)cidx[t]];
    } else if (f == CSR_ONE) {
        v = 1.0;
    }
    val[e] = (T)v;
}

template <typename T, int LANES>
__global__ void __launch_bounds__(VT) k_spmv(int64_t nrows, const int32_t* __restrict__ rp,
                                            const int32_t* __restrict__ col, const T* __restrict__ val,
                                            const T* __restrict__ x, T* __restrict__ y) {
    constexpr int U = 4;   // entries per lane whose loads are issued together
    const int64_t t = (int64_t)blockIdx.x * VT + threadIdx.x;
    const int64_t row = t / LANES;
    const int lane = (int)(t % LANES);
    T acc = T(0);
    if (row < nrows) {
        const int32_t b = rp[row], e = rp[row + 1];
        // lane entries k = b + lane + LANES j, summed in ascending j; U at a time: their column and
        // value loads first, then the U gathers of x, so a row costs two memory round trips per U
        // entries instead of two per entry
        for (int32_t k = b + lane; k < e; k += U * LANES) {
            int32_t c[U];
            T v[U], xv[U];
            // indices past the row's end are clamped to its last entry (loaded, not summed)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t kk = min(k + u * LANES, e - 1);
                c[u] = col[kk];
                v[u] = val[kk];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) xv[u] = x[c[u]];
#pragma unroll
            for (int u = 0; u < U; ++u) acc = k + u * LANES < e ? acc + v[u] * xv[u] : acc;
        }
    }
#pragma unroll
    for (int off = LANES / 2; off > 0; off >>= 1) acc += __shfl_down(acc, off, LANES);
    if (row < nrows && lane == 0) y[row] = acc;
}

unsigned blocks(int64_t n) { return (unsigned)((n + VT - 1) / VT); }

}  // namespace

void csr_elem_launch(int nloc, int64_t C, int n, int p, int L, const int32_t* map, const double* G,
                     const double* tab, int nq, const double* k, double* E, hipStream_t s) {
    switch (nloc) {
        case 4: hipLaunchKernelGGL(k_elem<4>, dim3(blocks(C)), dim3(VT), 0, s, C, n, p, L, map, G, tab, nq, k, E); break;
        case 10: hipLaunchKernelGGL(k_elem<10>, dim3(blocks(C)), dim3(VT), 0, s, C, n, p, L, map, G, tab, nq, k, E); break;
        default: hipLaunchKernelGGL(k_elem<20>, dim3(blocks(C)), dim3(VT), 0, s, C, n, p, L, map, G, tab, nq, k, E); break;
    }
}

template <typename T>
void csr_gather_launch(int64_t nnz, const int64_t* cptr, const int32_t* cidx, const uint8_t* flag, const double* E,
                       T* val, hipStream_t s) {
    hipLaunchKernelGGL((k_csr_gather<T>), dim3(blocks(nnz)), dim3(VT), 0, s, nnz, cptr, cidx, flag, E, val);
}
template void csr_gather_launch<double>(int64_t, const int64_t*, const int32_t*, const uint8_t*, const double*,
                                        double*, hipStream_t);
template void csr_gather_launch<float>(int64_t, const int64_t*, const int32_t*, const uint8_t*, const double*,
                                       float*, hipStream_t);

template <typename T>
void csr_spmv_launch(int64_t nrows, int lanes, const int32_t* rp, const int32_t* col, const T* val, const T* x, T* y,
                     hipStream_t s) {
    if (lanes <= 4)
        hipLaunchKernelGGL((k_spmv<T, 4>), dim3(blocks(nrows * 4)), dim3(VT), 0, s, nrows, rp, col, val, x, y);
    else if (lanes <= 8)
        hipLaunchKernelGGL((k_spmv<T, 8>), dim3(blocks(nrows * 8)), dim3(VT), 0, s, nrows, rp, col, val, x, y);
    else
        hipLaunchKernelGGL((k_spmv<T, 16>), dim3(blocks(nrows * 16)), dim3(VT), 0, s, nrows, rp, col, val, x, y);
}
template void csr_spmv_launch<double>(int64_t, int, const int32_t*, const int32_t*, const double*, const double*,
                                      double*, hipStream_t);
template void csr_spmv_launch<float>(int64_t, int, const int32_t*, const int32_t*, const float*, const float*,
                                     float*, hipStream_t);

}  // namespace fem
