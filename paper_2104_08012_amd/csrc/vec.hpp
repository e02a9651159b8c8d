// Launchers of the solver's vector and dense kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ops.hpp"

namespace fem {

template <typename T>
struct DotPairs {
    const T* x[3];
    const T* y[3];
};

// out[p] = sum_i x_p[i] y_p[i] for p < npair (npair <= 3), accumulated in FP64 with a fixed
// reduction order; partial holds dot_partial_doubles() doubles.
template <typename T>
void dot_launch(int npair, int64_t n, const DotPairs<T>& pr, double* partial, double* out, hipStream_t s);
size_t dot_partial_doubles();

// y = a x + b y (b = 0: y = a x, y not read)
template <typename T>
void axpby_launch(int64_t n, double a, const T* x, double b, T* y, hipStream_t s);

// CG scalars kept on the device (slots of the solver's scalar block), so that an iteration needs
// no host round trip: alpha = rz / pq; beta and rz <- rz_new; flag bits 1 (p^T A p <= 0) and
// 2 (r^T z <= 0) record breakdowns.
enum { CG_RZ = 8, CG_PQ = 9, CG_ALPHA = 10, CG_RR = 11, CG_FLAG = 12, CG_RZNEW = 13, CG_QZ = 14, CG_BETA = 15 };
void cg_update_dev_launch(int64_t n, const double* sc, const double* p, const double* q, double* x, double* r,
                          hipStream_t s);
// Fused forms with the reductions' fixed order (results bitwise those of the separate launches):
// sc[CG_PQ] = p^T q then alpha; x += alpha p, r -= alpha q and *rr = r^T r of the updated r;
// (sc[CG_RZNEW], sc[CG_QZ]) = (r^T z, q^T z) then beta.
void dot_alpha_launch(int64_t n, const double* p, const double* q, double* partial, double* sc, hipStream_t s);
void cg_update_dot_launch(int64_t n, const double* sc, const double* p, const double* q, double* x, double* r,
                          double* partial, double* rr, hipStream_t s);
void dot_beta_launch(int64_t n, const double* r, const double* z, const double* q, double* partial, double* sc,
                     bool flexible, hipStream_t s);
void cg_direction_dev_launch(int64_t n, const double* sc, const double* z, double* p, hipStream_t s);
// d = c1 d + c2 dinv r (first: d = c2 dinv r); x = d (init) or x += d
template <typename T>
void cheb_launch(int64_t n, double c1, double c2, const T* dinv, const T* r, T* d, T* x, bool first, bool init,
                 hipStream_t s);
template <typename A, typename B>
void cast_launch(int64_t n, const A* x, B* y, hipStream_t s);
template <typename T>
void fill_launch(int64_t n, T v, T* y, hipStream_t s);
template <typename T>
void recip_launch(int64_t n, const T* x, T* y, hipStream_t s);
template <typename T>
void mul_launch(int64_t n, const T* x, const T* sc, T* y, hipStream_t s);
template <typename T>
void div_launch(int64_t n, const T* x, const T* sc, T* y, hipStream_t s);
template <typename T>
void inject_launch(int nc, int stride, int nf, const double* kf, T* kc, hipStream_t s);
void random_launch(int64_t n, int L, uint64_t seed, double* v, hipStream_t s);
void probe_fill_launch(int L, int S, int c0, int c1, int c2, double* v, hipStream_t s);
void probe_extract_launch(int L, int p, int S, int c0, int c1, int c2, const double* y, double* A, hipStream_t s);
// In-place inverse of an n x n SPD matrix (row-major), kept in its lower 64 x 64 tiles (diagonal
// tiles whole; the strict upper tiles are left stale).  tmp: dense_invert_tmp_doubles(n) doubles.
size_t dense_invert_tmp_doubles(int64_t n);
fem_status dense_invert(int64_t n, double* A, double* tmp, hipStream_t s);
// Coarse inverse kept as the packed lower 64 x 64 tiles of its symmetric part; the solve reads
// each stored tile once (y_I += A_IJ x_J and y_J += A_IJ^T x_I through per-tile partials summed in
// a fixed order).  yl: lattice vector, boundary entries set to zero.
size_t sym_packed_doubles(int64_t n);   // entries of the packed tiles (FP64 or FP32 storage)
size_t sym_partial_doubles(int64_t n);
template <typename TA>
void sym_pack_launch(int64_t n, const double* A, TA* Ap, hipStream_t s);
template <typename TA>
void sym_solve_launch(int L, const TA* Ap, const double* xl, double* xc, double* part, double* yl,
                      hipStream_t s);

}  // namespace fem
