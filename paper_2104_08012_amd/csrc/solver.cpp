// Multigrid-preconditioned conjugate gradients (host orchestration of the device kernels).
//
// Method (paper Section 4 and Listing 2): a geometric multigrid cycle over the uniformly refined
// hierarchy, two Chebyshev iterations per level before and after the coarse correction, a direct
// solve on the coarsest level used, here as the preconditioner of CG on the finest level.
//   * Smoother: Chebyshev on D^-1 A over [lo, hi] * lambda_max (three-term recurrence of Saad,
//     Iterative Methods for Sparse Linear Systems, Alg. 12.1), the same polynomial before and after
//     the coarse correction so the cycle is symmetric; lambda_max from the largest Ritz value of a
//     few Lanczos steps on D^-1 A started from a counter-based random vector.
//   * Transfers: prolongation interpolates the coarse function at the fine nodes; restriction is
//     its transpose with boundary rows zeroed; level operators are rediscretised with the
//     coefficient injected at the coarse vertices.
//   * Coarsest level used: exact FP64 solve with the dense inverse of the interior block,
//     assembled by probing the matrix-free operator with (2p+1)^3 colour vectors, inverted by a
//     blocked Gauss-Jordan sweep on its lower triangle and kept as packed lower tiles (half the
//     bytes read per coarse solve).  When that level is too large for a dense inverse it is solved
//     by a nested FP64 MG-PCG over the levels below it, to a relative residual of coarse_rtol
//     (deepening the hierarchy under an expensive coarse level, as the paper does in Section 4).
//   * Outer CG in FP64: x0 given (usually 0), stop when the true residual satisfies
//     ||b - A x|| / ||b|| <= rtol.  Mixed precision keeps CG vectors, the outer operator, all
//     inner products and the coarse solve in FP64 and runs the smoother, the level residuals and
//     the transfers in FP32, casting at the entry and exit of the cycle and at the coarse level;
//     the Polak-Ribiere beta and periodic true-residual replacement make CG tolerant of the
//     slightly varying FP32 preconditioner.  Only the explicit FEM_COARSE_DENSE_F32 option stores
//     the dense coarse inverse in FP32 (its products still accumulate in FP64).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "vec.hpp"

using namespace fem;

namespace {

constexpr int64_t kDenseMax = 40000;   // interior dofs of a level inverted densely
constexpr int64_t kInnerDense = 8000;  // nested solve: its dense level, the finest at most this size

struct LevelWs {
    size_t x = 0, b = 0, r = 0, d = 0, dinv = 0, k64 = 0, k32 = 0, b64 = 0, x64 = 0;
    size_t patch = 0, pz = 0, patch_bytes = 0;   // star-patch smoother: buffer, B r
    size_t fb = 0, fx = 0;   // full multigrid: FP64 right-hand side and solution (below the top)
};

struct Layout {
    std::vector<LevelWs> lev;
    size_t cg_r = 0, cg_z = 0, cg_p = 0, cg_q = 0, partial = 0, scal = 0, dense = 0, dense_xc = 0, jac_diag = 0;
    size_t dense_packed = 0, dense_part = 0, dense_tmp = 0;
    size_t inner = 0, inner_bytes = 0;
    size_t total = 0;
    int top = 0, lo = 0, hi = 0, mixed = 0, nested = 0;
    int coarse32 = 0;   // dense inverse stored in FP32 (FEM_COARSE_DENSE_F32, mixed precision only)
    int64_t dense_n = 0;
};

int64_t interior_dofs(const fem_mesh& m, int l) {
    const int64_t M = m.lev[l].L - 2;
    return M * M * M;
}

int64_t interior_dofs(const fem_mesh& m, int l);

// Options of the nested coarse solver on levels 0..top: FP64 MG-PCG to coarse_rtol whose cycle
// stops at the finest level with at most kInnerDense interior dofs (solved with its dense inverse;
// a small dense solve is cheaper than the launch-bound smoothing of the levels below it).
fem_solve_opts inner_opts(const fem_mesh& m, const fem_solve_opts& o, int top) {
    fem_solve_opts in = o;
    in.rtol = o.coarse_rtol;
    in.max_it = 200;
    in.precision = FEM_PREC_FP64;
    int lo = 0;
    for (int l = top - 1; l >= 0; --l)
        if (interior_dofs(m, l) <= kInnerDense) {
            lo = l;
            break;
        }
    in.n_levels_used = top - lo + 1;
    in.coarse_method = FEM_COARSE_AUTO;
    in.replace_every = 0;
    in.flexible = 0;
    in.history = nullptr;
    in.history_cap = 0;
    in.preconditioner = FEM_PC_MG;
    in.smoother = FEM_SMOOTHER_JACOBI;
    return in;
}

// Workspace layout of a solver whose finest level is `top` (the mesh's finest for the public
// solver, the outer coarse level for a nested one).
fem_status make_layout(const fem_mesh& m, const fem_solve_opts& o, int top, Layout& L) {
    L.top = top;
    L.hi = top;
    const int avail = top + 1;
    const int used = (o.n_levels_used <= 0 || o.n_levels_used > avail) ? avail : o.n_levels_used;
    L.lo = top - used + 1;
    L.mixed = o.precision == FEM_PREC_MIXED;
    const size_t ts = L.mixed ? 4 : 8;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t r = off;
        off = align256(off + bytes);
        return r;
    };
    L.lev.assign(m.nlev, LevelWs{});
    for (int l = 0; l <= top; ++l) {
        const int64_t N = m.lev[l].N, NV = m.lev[l].NV;
        LevelWs& w = L.lev[l];
        w.k64 = take(NV * 8);
        if (L.mixed) w.k32 = take(NV * 4);
        if (l < L.lo) continue;
        w.x = take(N * ts);
        w.b = take(N * ts);
        w.r = take(N * ts);
        w.d = take(N * ts);
        w.dinv = take(N * ts);
        if (l > L.lo && o.smoother == FEM_SMOOTHER_PATCH) {
            w.patch_bytes = patch_bytes(m.lev[l], ts);
            w.patch = take(w.patch_bytes);
            w.pz = take(N * ts);
        }
        if (l == L.lo && L.mixed) {
            w.b64 = take(N * 8);
            w.x64 = take(N * 8);
        }
        if (l < top && o.preconditioner == FEM_PC_MG) {
            w.fb = take(N * 8);
            w.fx = take(N * 8);
        }
    }
    const int64_t Nf = m.lev[L.hi].N;
    L.cg_r = take(Nf * 8);
    L.cg_z = take(Nf * 8);
    L.cg_p = take(Nf * 8);
    L.cg_q = take(Nf * 8);
    L.partial = take(dot_partial_doubles() * 8);
    L.scal = take(64 * 8);
    if (o.preconditioner == FEM_PC_JACOBI) {
        L.jac_diag = take(Nf * 8);
        L.total = off;
        return FEM_OK;
    }
    const int64_t nI = interior_dofs(m, L.lo);
    const int method = o.coarse_method;
    const bool want_nested = method == FEM_COARSE_NESTED || (method == FEM_COARSE_AUTO && nI > kDenseMax);
    if (method == FEM_COARSE_DENSE_F32 && !L.mixed) {
        set_error("FP32 storage of the coarse inverse (FEM_COARSE_DENSE_F32) needs mixed precision");
        return FEM_ERR_INVALID_ARG;
    }
    if (want_nested && L.lo == 0) {
        if (method == FEM_COARSE_NESTED) {
            set_error("nested coarse solve needs a mesh level below the coarsest level used");
            return FEM_ERR_UNSUPPORTED;
        }
        set_error("coarsest mesh level has " + std::to_string(nI) + " interior dofs, more than the " +
                  std::to_string(kDenseMax) + " of the dense coarse solve; build the mesh with more refinements");
        return FEM_ERR_UNSUPPORTED;
    }
    if (!want_nested && nI > kDenseMax) {
        set_error("dense coarse solve limited to " + std::to_string(kDenseMax) + " interior dofs (level has " +
                  std::to_string(nI) + ")");
        return FEM_ERR_UNSUPPORTED;
    }
    L.nested = want_nested ? 1 : 0;
    if (L.nested) {
        Layout in;
        const fem_status st = make_layout(m, inner_opts(m, o, L.lo), L.lo, in);
        if (st) return st;
        L.inner = take(in.total);
        L.inner_bytes = in.total;
    } else {
        L.dense_n = nI;
        L.dense = take((size_t)nI * nI * 8);
        L.dense_xc = take(std::max<int64_t>(nI, 1) * 8);
        // the packed inverse: FP64 (an exact coarse solve in both precisions), or FP32 storage when
        // asked for explicitly (FEM_COARSE_DENSE_F32: half the bytes of the HBM-bound coarse
        // product, products still accumulated in FP64, the coarse correction then rounded like
        // the rest of the FP32 preconditioner)
        L.coarse32 = method == FEM_COARSE_DENSE_F32 ? 1 : 0;
        L.dense_packed = take(sym_packed_doubles(nI) * (L.coarse32 ? 4 : 8));
        L.dense_part = take(sym_partial_doubles(nI) * 8);
        L.dense_tmp = take(dense_invert_tmp_doubles(nI) * 8);
    }
    L.total = off;
    return FEM_OK;
}

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Largest eigenvalue of a small symmetric tridiagonal matrix (cyclic Jacobi on a dense copy).
double tridiag_max_eig(const std::vector<double>& a, const std::vector<double>& b) {
    const int n = (int)a.size();
    std::vector<double> A(n * n, 0.0);
    for (int i = 0; i < n; ++i) {
        A[i * n + i] = a[i];
        if (i + 1 < n) A[i * n + i + 1] = A[(i + 1) * n + i] = b[i];
    }
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) off += A[i * n + j] * A[i * n + j];
        if (off < 1e-30) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = A[p * n + q];
                if (std::fabs(apq) < 1e-300) continue;
                const double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {
                    const double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - s * akq;
                    A[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    const double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - s * aqk;
                    A[q * n + k] = s * apk + c * aqk;
                }
            }
    }
    double mx = -1e300;
    for (int i = 0; i < n; ++i) mx = std::max(mx, A[i * n + i]);
    return mx;
}

// Event and free calls whose failure leaves nothing to undo.
void ignore(hipError_t) {}

}  // namespace

#define FEM_TRY(expr)                   \
    do {                                \
        const fem_status _st = (expr);  \
        if (_st != FEM_OK) return _st;  \
    } while (0)

struct fem_solver {
    const fem_mesh* m = nullptr;
    fem_solve_opts o{};
    char* ws = nullptr;
    size_t ws_bytes = 0;
    Layout L;
    bool kvar = false;
    bool ready = false;
    std::vector<double> lmax;
    double* hscal = nullptr;   // pinned host scalars
    hipStream_t s = nullptr;
    double coarse_ms = 0.0;
    std::vector<double> level_ms;
    int coarse_iters = 0;
    // two sets (alternate iterations) of per-level events: pre start/end, post start/end; coarse
    // start/end; then the event marking each iteration's residual copy
    std::vector<hipEvent_t> ev;
    int evset = 0;
    int ev_per_set() const { return 4 * m->nlev + 2; }
    hipEvent_t* evs(int set) { return &ev[(size_t)set * ev_per_set()]; }
    bool timing = false;   // per-level events (fem_solve_opts.level_timing)
    std::unique_ptr<fem_solver> inner;   // nested coarse solver over levels 0..L.lo

    ~fem_solver() {
        for (auto& e : ev) ignore(hipEventDestroy(e));
        if (hscal) ignore(hipHostFree(hscal));
    }

    template <typename T>
    T* p(size_t off) const { return reinterpret_cast<T*>(ws + off); }

    fem_status init(const fem_mesh* mesh, const fem_solve_opts& opts, int top, char* wsp, size_t bytes);

    fem_status apply64(int l, const double* x, double alpha, const double* z, double beta, double* y) {
        ScatterIO<double> io;
        io.x = x;
        io.k = kvar ? p<double>(L.lev[l].k64) : nullptr;
        io.y = y;
        io.z = z;
        io.alpha = alpha;
        io.beta = beta;
        io.row_mode = ROW_IDENTITY;
        io.xid = x;
        io.mask_cols = 1;
        return run_scatter<double>(*m, l, K_APPLY, kvar, io, s);
    }
    template <typename T>
    fem_status applyT(int l, const T* x, double alpha, const T* z, double beta, T* y);

    fem_status dots(int npair, int64_t n, const double* x0, const double* y0, const double* x1, const double* y1,
                    double* out) {
        DotPairs<double> pr{{x0, x1, nullptr}, {y0, y1, nullptr}};
        dot_launch<double>(npair, n, pr, p<double>(L.partial), p<double>(L.scal), s);
        hipError_t e = hipMemcpyAsync(hscal, p<double>(L.scal), npair * sizeof(double), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            set_error(std::string("solver reduction: ") + hipGetErrorString(e));
            return FEM_ERR_HIP;
        }
        for (int i = 0; i < npair; ++i) out[i] = hscal[i];
        return FEM_OK;
    }
    fem_status dot(int64_t n, const double* x, const double* y, double& out) {
        double o2[2];
        FEM_TRY(dots(1, n, x, y, nullptr, nullptr, o2));
        out = o2[0];
        return FEM_OK;
    }

    template <typename T>
    fem_status vcycle(int l, const T* b, T* x);
    fem_status coarse_solve(const double* b64, double* x64);
    fem_status setup(const double* k_top);
    fem_status lanczos(int l, double& lm);
    fem_status lanczos_patch(int l, double& lm);
    fem_status patch64(int l, const double* x, double* y);
    fem_status precondition(const double* r, double* z);
    fem_status cg(const double* b, double* x, int& iters, double& rel_true, bool& converged, bool x_zero = false);
    fem_status fmg(const double* b, double* x, double& rel_true);
    void accumulate_times(int set);
};

fem_status fem_solver::init(const fem_mesh* mesh, const fem_solve_opts& opts, int top, char* wsp, size_t bytes) {
    m = mesh;
    o = opts;
    FEM_TRY(make_layout(*m, o, top, L));
    if (bytes < L.total) {
        set_error("solver workspace smaller than fem_solve_workspace_bytes");
        return FEM_ERR_WORKSPACE;
    }
    ws = wsp;
    ws_bytes = bytes;
    if (hipHostMalloc((void**)&hscal, 64 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        hscal = nullptr;
        set_error("solver: pinned host allocation failed");
        return FEM_ERR_HIP;
    }
    const int nl = m->nlev;
    ev.assign(2 * (4 * nl + 2) + 1, nullptr);
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            e = nullptr;
            set_error("solver: event creation failed");
            return FEM_ERR_HIP;
        }
    level_ms.assign(nl, 0.0);
    timing = o.level_timing != 0;
    if (L.nested) {
        inner.reset(new fem_solver());
        FEM_TRY(inner->init(m, inner_opts(*m, o, L.lo), L.lo, ws + L.inner, L.inner_bytes));
        inner->timing = false;
    }
    return FEM_OK;
}

template <>
fem_status fem_solver::applyT<double>(int l, const double* x, double alpha, const double* z, double beta, double* y) {
    return apply64(l, x, alpha, z, beta, y);
}
template <>
fem_status fem_solver::applyT<float>(int l, const float* x, double alpha, const float* z, double beta, float* y) {
    ScatterIO<float> io;
    io.x = x;
    io.k = kvar ? p<float>(L.lev[l].k32) : nullptr;
    io.y = y;
    io.z = z;
    io.alpha = alpha;
    io.beta = beta;
    io.row_mode = ROW_IDENTITY;
    io.xid = x;
    io.mask_cols = 1;
    return run_scatter<float>(*m, l, K_APPLY, kvar, io, s);
}

// x64 = A_lo^-1 b64 on the coarsest level used (dense inverse, or nested MG-PCG from x = 0).
fem_status fem_solver::coarse_solve(const double* b64, double* x64) {
    if (inner) {
        inner->s = s;
        fill_launch<double>(m->lev[L.lo].N, 0.0, x64, s);
        int its = 0;
        double rel = 0.0;
        bool conv = false;
        FEM_TRY(inner->cg(b64, x64, its, rel, conv, true));
        coarse_iters += its;
        if (!conv) {
            set_error("nested coarse solve stopped at relative residual " + std::to_string(rel) + " > coarse_rtol");
            return FEM_ERR_BREAKDOWN;
        }
        return FEM_OK;
    }
    const HostLevel& C = m->lev[L.lo];
    if (L.coarse32)
        sym_solve_launch(C.L, p<float>(L.dense_packed), b64, p<double>(L.dense_xc), p<double>(L.dense_part), x64, s);
    else
        sym_solve_launch(C.L, p<double>(L.dense_packed), b64, p<double>(L.dense_xc), p<double>(L.dense_part), x64, s);
    return check_launch("coarse solve");
}

template <typename T>
fem_status fem_solver::vcycle(int l, const T* b, T* x) {
    const int nl = (int)m->lev.size();
    hipEvent_t* ev0 = evs(evset);
    hipEvent_t* e = timing ? &ev0[4 * l] : nullptr;
    if (l == L.lo) {
        if (timing) ignore(hipEventRecord(ev0[4 * nl], s));
        if (L.mixed) {
            const int64_t n = m->lev[l].N;
            cast_launch<T, double>(n, b, p<double>(L.lev[l].b64), s);
            FEM_TRY(coarse_solve(p<double>(L.lev[l].b64), p<double>(L.lev[l].x64)));
            cast_launch<double, T>(n, p<double>(L.lev[l].x64), x, s);
        } else {
            FEM_TRY(coarse_solve(reinterpret_cast<const double*>(b), reinterpret_cast<double*>(x)));
        }
        if (timing) ignore(hipEventRecord(ev0[4 * nl + 1], s));
        return FEM_OK;
    }
    const HostLevel& H = m->lev[l];
    const int64_t n = H.N;
    const LevelWs& w = L.lev[l];
    T* r = p<T>(w.r);
    T* d = p<T>(w.d);
    const T* dinv = p<T>(w.dinv);
    const int deg = std::max(1, o.cheb_degree);
    const double lm = lmax[l];
    const double a = o.cheb_lo * lm, bb = o.cheb_hi * lm;
    const double theta = 0.5 * (bb + a), delta = 0.5 * (bb - a), sigma = theta / delta;
    if (timing) ignore(hipEventRecord(e[0], s));
    // one Chebyshev step d = c1 d + c2 B src, x (+)= d, with B = D^-1 or the star patches
    auto cheb = [&](double c1, double c2, const T* src, bool first, bool init) -> fem_status {
        if (o.smoother == FEM_SMOOTHER_PATCH) {
            T* pz = p<T>(w.pz);
            FEM_TRY(patch_apply<T>(*m, l, p<char>(w.patch), src, pz, s));
            cheb_launch<T>(n, c1, c2, static_cast<const T*>(nullptr), pz, d, x, first, init, s);
        } else {
            cheb_launch<T>(n, c1, c2, dinv, src, d, x, first, init, s);
        }
        return FEM_OK;
    };
    // pre-smoothing from x = 0; r tracks b - A x
    double rho = 1.0 / sigma;
    FEM_TRY(cheb(0.0, 1.0 / theta, b, true, true));
    FEM_TRY(applyT<T>(l, d, -1.0, b, 1.0, r));
    for (int k = 1; k < deg; ++k) {
        const double rn = 1.0 / (2.0 * sigma - rho);
        FEM_TRY(cheb(rn * rho, 2.0 * rn / delta, r, false, false));
        rho = rn;
        FEM_TRY(applyT<T>(l, d, -1.0, r, 1.0, r));
    }
    // coarse-grid correction
    T* bc = p<T>(L.lev[l - 1].b);
    T* xc = p<T>(L.lev[l - 1].x);
    FEM_TRY(run_restrict<T>(*m, l, r, bc, s));
    if (timing) ignore(hipEventRecord(e[1], s));
    FEM_TRY(vcycle<T>(l - 1, bc, xc));
    if (timing) ignore(hipEventRecord(e[2], s));
    FEM_TRY(run_prolong<T>(*m, l, xc, x, s));
    // post-smoothing from x
    FEM_TRY(applyT<T>(l, x, -1.0, b, 1.0, r));
    rho = 1.0 / sigma;
    FEM_TRY(cheb(0.0, 1.0 / theta, r, true, false));
    for (int k = 1; k < deg; ++k) {
        FEM_TRY(applyT<T>(l, d, -1.0, r, 1.0, r));
        const double rn = 1.0 / (2.0 * sigma - rho);
        FEM_TRY(cheb(rn * rho, 2.0 * rn / delta, r, false, false));
        rho = rn;
    }
    if (timing) ignore(hipEventRecord(e[3], s));
    return FEM_OK;
}

// Largest Ritz value of o.eig_iters Lanczos steps on D^-1 A in the D inner product (FP64, using
// the four FP64 CG vectors as scratch: v, w, v_prev and the diagonal D).
fem_status fem_solver::lanczos(int l, double& lm) {
    const HostLevel& H = m->lev[l];
    const int64_t n = H.N;
    double* v = p<double>(L.cg_r);
    double* wv = p<double>(L.cg_z);
    double* vp = p<double>(L.cg_p);
    double* dg = p<double>(L.cg_q);
    {
        ScatterIO<double> io;
        io.k = kvar ? p<double>(L.lev[l].k64) : nullptr;
        io.y = dg;
        io.row_mode = ROW_ONE;
        FEM_TRY(run_scatter<double>(*m, l, K_DIAG, kvar, io, s));
    }
    random_launch(n, H.L, 0x5eed0005ull + (uint64_t)l, v, s);
    fill_launch<double>(n, 0.0, vp, s);
    double nv = 0.0;
    mul_launch<double>(n, v, dg, wv, s);
    FEM_TRY(dot(n, v, wv, nv));
    if (!(nv > 0)) {
        set_error("Lanczos start vector has zero D-norm");
        return FEM_ERR_BREAKDOWN;
    }
    axpby_launch<double>(n, 0.0, v, 1.0 / std::sqrt(nv), v, s);
    std::vector<double> al, be;
    double beta = 0.0;
    const int steps = std::max(2, o.eig_iters);
    for (int it = 0; it < steps; ++it) {
        FEM_TRY(apply64(l, v, 1.0, nullptr, 0.0, wv));                // w = A v
        double alpha = 0.0;
        FEM_TRY(dot(n, wv, v, alpha));                                 // (D^-1 A v)^T D v
        al.push_back(alpha);
        div_launch<double>(n, wv, dg, wv, s);                          // w = D^-1 A v
        axpby_launch<double>(n, -alpha, v, 1.0, wv, s);
        if (beta != 0.0) axpby_launch<double>(n, -beta, vp, 1.0, wv, s);
        mul_launch<double>(n, wv, dg, vp, s);                          // v_prev is free here
        double b2 = 0.0;
        FEM_TRY(dot(n, wv, vp, b2));
        if (!(b2 > 0) || it == steps - 1) break;
        beta = std::sqrt(b2);
        be.push_back(beta);
        axpby_launch<double>(n, 1.0, v, 0.0, vp, s);                   // v_prev = v
        axpby_launch<double>(n, 1.0 / beta, wv, 0.0, v, s);            // v = w / beta
    }
    be.resize(al.size() > 0 ? al.size() - 1 : 0);
    lm = tridiag_max_eig(al, be);
    if (!std::isfinite(lm) || lm <= 0) {
        set_error("Lanczos estimate of lambda_max failed");
        return FEM_ERR_BREAKDOWN;
    }
    return FEM_OK;
}

// y = B_patch x on level l in FP64 (the FP32-stored patches of a mixed solver through the
// level's FP32 vectors).
fem_status fem_solver::patch64(int l, const double* x, double* y) {
    const LevelWs& w = L.lev[l];
    if (!L.mixed) return patch_apply<double>(*m, l, p<char>(w.patch), x, y, s);
    const int64_t n = m->lev[l].N;
    cast_launch<double, float>(n, x, p<float>(w.r), s);
    FEM_TRY(patch_apply<float>(*m, l, p<char>(w.patch), p<float>(w.r), p<float>(w.pz), s));
    cast_launch<float, double>(n, p<float>(w.pz), y, s);
    return FEM_OK;
}

// Largest eigenvalue estimate of B_patch A from o.eig_iters steps of preconditioned CG on A e = v
// (v the seeded random start): the CG coefficients alpha_j, beta_j give the Lanczos tridiagonal
// of B A with diagonal 1/alpha_j + beta_{j-1}/alpha_{j-1} and off-diagonal sqrt(beta_j)/alpha_j
// (the CG-Lanczos relation; Saad, Iterative Methods for Sparse Linear Systems, 6.7.3).
fem_status fem_solver::lanczos_patch(int l, double& lm) {
    const int64_t n = m->lev[l].N;
    double* r = p<double>(L.cg_r);
    double* z = p<double>(L.cg_z);
    double* pv = p<double>(L.cg_p);
    double* q = p<double>(L.cg_q);
    random_launch(n, m->lev[l].L, 0x5eed0005ull + (uint64_t)l, r, s);
    FEM_TRY(patch64(l, r, z));
    cast_launch<double, double>(n, z, pv, s);
    double rz = 0.0;
    FEM_TRY(dot(n, r, z, rz));
    if (!(rz > 0)) {
        set_error("CG-Lanczos start vector has zero preconditioned norm");
        return FEM_ERR_BREAKDOWN;
    }
    std::vector<double> al, be;
    const int steps = std::max(2, o.eig_iters);
    for (int it = 0; it < steps; ++it) {
        FEM_TRY(apply64(l, pv, 1.0, nullptr, 0.0, q));               // q = A p
        double pq = 0.0;
        FEM_TRY(dot(n, pv, q, pq));
        if (!(pq > 0)) break;
        al.push_back(rz / pq);
        if (it == steps - 1) break;
        axpby_launch<double>(n, -al.back(), q, 1.0, r, s);           // r -= alpha q
        FEM_TRY(patch64(l, r, z));                                   // z = B r
        double rz2 = 0.0;
        FEM_TRY(dot(n, r, z, rz2));
        if (!(rz2 > 0)) break;
        be.push_back(rz2 / rz);
        rz = rz2;
        axpby_launch<double>(n, 1.0, z, be.back(), pv, s);           // p = z + beta p
    }
    const size_t k = al.size();
    if (k == 0) {
        set_error("CG-Lanczos estimate of lambda_max failed");
        return FEM_ERR_BREAKDOWN;
    }
    std::vector<double> dg(k), off(k - 1);
    for (size_t j = 0; j < k; ++j) dg[j] = 1.0 / al[j] + (j > 0 ? be[j - 1] / al[j - 1] : 0.0);
    for (size_t j = 0; j + 1 < k; ++j) off[j] = std::sqrt(be[j]) / al[j];
    lm = tridiag_max_eig(dg, off);
    if (!std::isfinite(lm) || lm <= 0) {
        set_error("CG-Lanczos estimate of lambda_max failed");
        return FEM_ERR_BREAKDOWN;
    }
    return FEM_OK;
}

// k_top: the coefficient on the vertex lattice of this solver's finest level (NULL for k = 1).
fem_status fem_solver::setup(const double* k_top) {
    kvar = k_top != nullptr;
    const int nl = m->nlev, top = L.top;
    lmax.assign(nl, 0.0);
    // coefficient on every level by injection
    if (kvar) {
        for (int l = 0; l <= top; ++l) {
            const int stride = 1 << (top - l);
            inject_launch<double>(m->lev[l].n, stride, m->lev[top].n, k_top, p<double>(L.lev[l].k64), s);
            if (L.mixed) inject_launch<float>(m->lev[l].n, stride, m->lev[top].n, k_top, p<float>(L.lev[l].k32), s);
        }
    }
    if (o.preconditioner == FEM_PC_JACOBI) {
        ScatterIO<double> io;
        io.k = kvar ? p<double>(L.lev[top].k64) : nullptr;
        io.y = p<double>(L.jac_diag);
        io.row_mode = ROW_ONE;
        FEM_TRY(run_scatter<double>(*m, top, K_DIAG, kvar, io, s));
    } else {
        // Jacobi scaling per smoothed level
        for (int l = L.lo + 1; l <= L.hi; ++l) {
            const int64_t n = m->lev[l].N;
            double* dg = p<double>(L.cg_q);
            ScatterIO<double> io;
            io.k = kvar ? p<double>(L.lev[l].k64) : nullptr;
            io.y = dg;
            io.row_mode = ROW_ONE;
            FEM_TRY(run_scatter<double>(*m, l, K_DIAG, kvar, io, s));
            if (L.mixed) {
                recip_launch<double>(n, dg, dg, s);
                cast_launch<double, float>(n, dg, p<float>(L.lev[l].dinv), s);
            } else {
                recip_launch<double>(n, dg, p<double>(L.lev[l].dinv), s);
            }
        }
        // star-patch smoother: the inverses of the vertex stars per smoothed level
        if (o.smoother == FEM_SMOOTHER_PATCH)
            for (int l = L.lo + 1; l <= L.hi; ++l) {
                const double* kl = kvar ? p<double>(L.lev[l].k64) : nullptr;
                if (L.mixed) FEM_TRY(patch_setup<float>(*m, l, kl, p<char>(L.lev[l].patch), s));
                else FEM_TRY(patch_setup<double>(*m, l, kl, p<char>(L.lev[l].patch), s));
            }
        // lambda_max per smoothed level
        for (int l = L.lo + 1; l <= L.hi; ++l) {
            if (o.lambda_max_override && o.lambda_max_override[l] > 0) lmax[l] = o.lambda_max_override[l];
            else if (o.smoother == FEM_SMOOTHER_PATCH) FEM_TRY(lanczos_patch(l, lmax[l]));
            else FEM_TRY(lanczos(l, lmax[l]));
        }
        if (inner) {
            inner->s = s;
            FEM_TRY(inner->setup(kvar ? p<double>(L.lev[L.lo].k64) : nullptr));
            for (int l = 0; l <= L.lo; ++l) lmax[l] = inner->lmax[l];
        } else {
            // coarse operator: dense interior block by probing, then its inverse
            const HostLevel& C = m->lev[L.lo];
            const int P = C.p, S = 2 * P + 1;
            double* A = p<double>(L.dense);
            const int64_t nd = L.dense_n;
            fill_launch<double>(nd * nd, 0.0, A, s);
            double* v = p<double>(L.cg_r);
            double* y = p<double>(L.cg_z);
            for (int c2 = 0; c2 < S; ++c2)
                for (int c1 = 0; c1 < S; ++c1)
                    for (int c0 = 0; c0 < S; ++c0) {
                        probe_fill_launch(C.L, S, c0, c1, c2, v, s);
                        FEM_TRY(apply64(L.lo, v, 1.0, nullptr, 0.0, y));
                        probe_extract_launch(C.L, P, S, c0, c1, c2, y, A, s);
                    }
            FEM_TRY(dense_invert(nd, A, p<double>(L.dense_tmp), s));
            if (L.coarse32) sym_pack_launch(nd, A, p<float>(L.dense_packed), s);
            else sym_pack_launch(nd, A, p<double>(L.dense_packed), s);
        }
    }
    const hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        set_error(std::string("solver setup: ") + hipGetErrorString(e));
        return FEM_ERR_HIP;
    }
    FEM_TRY(check_launch("solver setup"));
    ready = true;
    return FEM_OK;
}

// Adds the per-level times of a completed V-cycle whose events are in the given set.
void fem_solver::accumulate_times(int set) {
    const int nl = m->nlev;
    hipEvent_t* e = evs(set);
    for (int l = L.lo + 1; l <= L.hi; ++l) {
        float a = 0.f, b = 0.f;
        if (hipEventElapsedTime(&a, e[4 * l], e[4 * l + 1]) == hipSuccess &&
            hipEventElapsedTime(&b, e[4 * l + 2], e[4 * l + 3]) == hipSuccess)
            level_ms[l] += a + b;
    }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e[4 * nl], e[4 * nl + 1]) == hipSuccess) {
        coarse_ms += ms;
        level_ms[L.lo] += ms;
    }
}

fem_status fem_solver::precondition(const double* r, double* z) {
    const int hi = L.hi;
    if (o.preconditioner == FEM_PC_JACOBI) {
        div_launch<double>(m->lev[hi].N, r, p<double>(L.jac_diag), z, s);
        return check_launch("Jacobi preconditioner");
    }
    if (L.mixed) {
        const int64_t n = m->lev[hi].N;
        float* b = p<float>(L.lev[hi].b);
        float* x = p<float>(L.lev[hi].x);
        cast_launch<double, float>(n, r, b, s);
        FEM_TRY(vcycle<float>(hi, b, x));
        cast_launch<float, double>(n, x, z, s);
        return FEM_OK;
    }
    return vcycle<double>(hi, r, z);
}

// Preconditioned CG on this solver's finest level; x holds the initial guess and returns the
// iterate (x_zero: the guess is known to be zero, so r = b).  converged reports whether the true
// relative residual reached o.rtol.
//
// The scalars alpha, beta and r^T z stay on the device.  Each iteration enqueues q = A p, alpha,
// the update of x and r, r^T r (copied to pinned host memory behind an event) and then,
// speculatively, the preconditioner, r^T z, beta and the new direction; the host waits only for
// that iteration's r^T r, which is ready before the preconditioner runs, so the queue never
// drains.  On convergence the speculative work is discarded (it touches only z, p and scalars).
fem_status fem_solver::cg(const double* b, double* x, int& it, double& rel_true, bool& converged, bool x_zero) {
    const int hi = L.hi;
    const int64_t n = m->lev[hi].N;
    double* r = p<double>(L.cg_r);
    double* z = p<double>(L.cg_z);
    double* pp = p<double>(L.cg_p);
    double* q = p<double>(L.cg_q);
    double* sc = p<double>(L.scal);
    double* part = p<double>(L.partial);
    it = 0;
    converged = false;
    rel_true = 0.0;
    auto record = [&](int i, double v) {
        if (o.history && i < o.history_cap) o.history[i] = v;
    };
    auto dotdev = [&](int npair, const double* x0, const double* y0, const double* x1, const double* y1, int slot) {
        DotPairs<double> pr{{x0, x1, nullptr}, {y0, y1, nullptr}};
        dot_launch<double>(npair, n, pr, part, sc + slot, s);
    };
    const bool tmg = timing && o.preconditioner == FEM_PC_MG;
    double bb = 0.0, rr = 0.0;
    FEM_TRY(dot(n, b, b, bb));
    const double nb = std::sqrt(bb);
    if (!std::isfinite(nb)) {
        set_error("solver: right-hand side is not finite");
        return FEM_ERR_BREAKDOWN;
    }
    if (nb == 0.0) {
        fill_launch<double>(n, 0.0, x, s);
        record(0, 0.0);
        converged = true;
        return check_launch("solver");
    }
    if (x_zero) {
        axpby_launch<double>(n, 1.0, b, 0.0, r, s);              // r = b
        rr = bb;
    } else {
        FEM_TRY(apply64(hi, x, -1.0, b, 1.0, r));             // r = b - A x
        FEM_TRY(dot(n, r, r, rr));
    }
    double rel = std::sqrt(rr) / nb;
    double rel_checked = -1.0;   // true relative residual of the current x, once computed
    record(0, rel);
    // z = B r, rz, p = z (also the restart after a failed true-residual check)
    auto start = [&]() -> fem_status {
        evset = 0;
        FEM_TRY(precondition(r, z));
        double rz = 0.0;
        FEM_TRY(dot(n, r, z, rz));
        if (tmg) accumulate_times(0);
        if (!(rz > 0) || !std::isfinite(rz)) {
            set_error("solver: preconditioner is not positive definite (r^T B r <= 0)");
            return FEM_ERR_BREAKDOWN;
        }
        fill_launch<double>(1, rz, sc + CG_RZ, s);
        fill_launch<double>(1, 0.0, sc + CG_FLAG, s);
        axpby_launch<double>(n, 1.0, z, 0.0, pp, s);
        return FEM_OK;
    };
    if (rel <= o.rtol) {
        converged = true;
        rel_checked = rel;
    } else {
        FEM_TRY(start());
    }
    hipEvent_t done = ev.back();
    bool pending_times = false;
    // next search direction: z = B r, r^T z and q^T z (q = A p), beta, p = z + beta p
    auto tail = [&](int set) -> fem_status {
        evset = set;
        FEM_TRY(precondition(r, z));
        dot_beta_launch(n, r, z, q, part, sc, o.flexible != 0, s);
        cg_direction_dev_launch(n, sc, z, pp, s);
        return FEM_OK;
    };
    while (!converged && it < o.max_it) {
        FEM_TRY(apply64(hi, pp, 1.0, nullptr, 0.0, q));        // q = A p
        dot_alpha_launch(n, pp, q, part, sc, s);
        ++it;
        if (o.replace_every > 0 && it % o.replace_every == 0) {
            // residual replacement: r^T r of the true residual
            cg_update_dev_launch(n, sc, pp, q, x, r, s);
            FEM_TRY(apply64(hi, x, -1.0, b, 1.0, r));
            dotdev(1, r, r, nullptr, nullptr, CG_RR);
        } else {
            cg_update_dot_launch(n, sc, pp, q, x, r, part, sc + CG_RR, s);
        }
        hipError_t e = hipMemcpyAsync(hscal, sc + CG_RR, 2 * sizeof(double), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipEventRecord(done, s);
        // far from convergence the next direction is computed speculatively, before the residual
        // is known on the host; close to it the host checks first
        const int set = it & 1;
        const bool spec = rel > 30.0 * o.rtol;
        if (spec) FEM_TRY(tail(set));
        if (e == hipSuccess) e = hipEventSynchronize(done);
        if (e != hipSuccess) {
            set_error(std::string("solver: ") + hipGetErrorString(e));
            return FEM_ERR_HIP;
        }
        if (tmg && pending_times) accumulate_times(set ^ 1);   // the previous iteration's V-cycle
        pending_times = false;
        rr = hscal[0];
        const int flag = (int)hscal[1];
        if (flag) {
            set_error(flag & 1 ? "solver: CG breakdown (p^T A p <= 0 or not finite)"
                               : "solver: preconditioner is not positive definite (r^T B r <= 0)");
            return FEM_ERR_BREAKDOWN;
        }
        rel = std::sqrt(rr) / nb;
        record(it, rel);
        if (!std::isfinite(rel)) {
            set_error("solver: residual not finite");
            return FEM_ERR_BREAKDOWN;
        }
        if (rel <= o.rtol) {
            // confirm with the true residual (stream-ordered after any speculative work)
            FEM_TRY(apply64(hi, x, -1.0, b, 1.0, q));
            double tt = 0.0;
            FEM_TRY(dot(n, q, q, tt));
            if (tmg && spec) accumulate_times(set);
            if (std::sqrt(tt) / nb <= o.rtol) {
                converged = true;
                rel_checked = std::sqrt(tt) / nb;
                break;
            }
            if (spec) {
                // the speculative direction used the recurrence residual: restart from the true one
                axpby_launch<double>(n, 1.0, q, 0.0, r, s);
                FEM_TRY(start());
                continue;
            }
            // continue from the true residual; q must hold A p again for the Polak-Ribiere beta
            axpby_launch<double>(n, 1.0, q, 0.0, r, s);
            FEM_TRY(apply64(hi, pp, 1.0, nullptr, 0.0, q));
        }
        if (!spec) FEM_TRY(tail(set));
        pending_times = tmg;
    }
    if (pending_times) {
        const hipError_t e = hipStreamSynchronize(s);
        if (e == hipSuccess) accumulate_times(evset);
    }
    // true residual at exit (already known when the loop stopped on its check)
    if (rel_checked >= 0.0) {
        rel_true = rel_checked;
        return check_launch("solver");
    }
    FEM_TRY(apply64(hi, x, -1.0, b, 1.0, q));
    double tt = 0.0;
    FEM_TRY(dot(n, q, q, tt));
    rel_true = std::sqrt(tt) / nb;
    if (!converged) converged = rel_true <= o.rtol;
    return FEM_OK;
}

// One full-multigrid cycle (see fem_solver_fmg in the header).
fem_status fem_solver::fmg(const double* b, double* x, double& rel_true) {
    const int hi = L.hi, lo = L.lo;
    auto fb = [&](int l) -> double* { return l == hi ? const_cast<double*>(b) : p<double>(L.lev[l].fb); };
    auto fx = [&](int l) -> double* { return l == hi ? x : p<double>(L.lev[l].fx); };
    for (int l = hi; l > lo; --l) {
        FEM_TRY(run_restrict<double>(*m, l, fb(l), fb(l - 1), s));
    }
    FEM_TRY(coarse_solve(fb(lo), fx(lo)));                    // FP64 in both precisions
    for (int l = lo + 1; l <= hi; ++l) {
        const int64_t n = m->lev[l].N;
        fill_launch<double>(n, 0.0, fx(l), s);
        FEM_TRY(run_prolong<double>(*m, l, fx(l - 1), fx(l), s));
        if (L.mixed) {
            double* r64 = p<double>(L.cg_q);
            double* e64 = p<double>(L.cg_z);
            FEM_TRY(apply64(l, fx(l), -1.0, fb(l), 1.0, r64));
            cast_launch<double, float>(n, r64, p<float>(L.lev[l].b), s);
            FEM_TRY(vcycle<float>(l, p<float>(L.lev[l].b), p<float>(L.lev[l].x)));
            cast_launch<float, double>(n, p<float>(L.lev[l].x), e64, s);
            axpby_launch<double>(n, 1.0, e64, 1.0, fx(l), s);
        } else {
            FEM_TRY(apply64(l, fx(l), -1.0, fb(l), 1.0, p<double>(L.lev[l].b)));
            FEM_TRY(vcycle<double>(l, p<double>(L.lev[l].b), p<double>(L.lev[l].x)));
            axpby_launch<double>(n, 1.0, p<double>(L.lev[l].x), 1.0, fx(l), s);
        }
    }
    const int64_t n = m->lev[hi].N;
    double* q = p<double>(L.cg_q);
    FEM_TRY(apply64(hi, x, -1.0, b, 1.0, q));
    double bb = 0.0, qq = 0.0;
    FEM_TRY(dot(n, b, b, bb));
    FEM_TRY(dot(n, q, q, qq));
    rel_true = bb > 0 ? std::sqrt(qq / bb) : std::sqrt(qq);
    return FEM_OK;
}

extern "C" {

void fem_solve_opts_default(fem_solve_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->rtol = 1e-8;
    o->max_it = 200;
    o->precision = FEM_PREC_FP64;
    o->n_levels_used = 0;
    o->cheb_degree = 2;
    o->cheb_lo = 0.1;
    o->cheb_hi = 1.1;
    o->eig_iters = 10;
    o->coarse_method = FEM_COARSE_AUTO;
    o->lambda_max_override = nullptr;
    o->coarse_rtol = 1e-10;
    o->replace_every = 25;
    o->flexible = 0;
    o->history = nullptr;
    o->history_cap = 0;
    o->preconditioner = FEM_PC_MG;
    o->level_timing = 0;
    o->smoother = FEM_SMOOTHER_JACOBI;
}

static fem_status check_opts(const fem_mesh* m, const fem_solve_opts* o) {
    if (!m || !o) {
        set_error("solver: NULL mesh or options");
        return FEM_ERR_INVALID_ARG;
    }
    if (!(o->rtol > 0) || o->max_it < 1 || o->cheb_degree < 1 || o->cheb_degree > 16 || !(o->cheb_hi > o->cheb_lo) ||
        !(o->cheb_lo > 0) || (o->precision != FEM_PREC_FP64 && o->precision != FEM_PREC_MIXED) ||
        o->n_levels_used < 0 || o->eig_iters < 0 || o->eig_iters > 64 || !(o->coarse_rtol > 0) ||
        o->coarse_method < FEM_COARSE_AUTO || o->coarse_method > FEM_COARSE_DENSE_F32 ||
        (o->preconditioner != FEM_PC_MG && o->preconditioner != FEM_PC_JACOBI) ||
        (o->smoother != FEM_SMOOTHER_JACOBI && o->smoother != FEM_SMOOTHER_PATCH)) {
        set_error("solver: invalid options");
        return FEM_ERR_INVALID_ARG;
    }
    if (o->smoother == FEM_SMOOTHER_PATCH) {
        std::string why;
        for (int l = 0; l < m->nlev; ++l)
            if (!patch_supported(m->lev[l], why)) {
                set_error("solver: star-patch smoother: " + why);
                return FEM_ERR_UNSUPPORTED;
            }
    }
    return FEM_OK;
}

fem_status fem_solve_workspace_bytes(const fem_mesh* m, const fem_solve_opts* o, size_t* bytes) {
    fem_status st = check_opts(m, o);
    if (st) return st;
    if (!bytes) {
        set_error("fem_solve_workspace_bytes: NULL output");
        return FEM_ERR_INVALID_ARG;
    }
    Layout L;
    st = make_layout(*m, *o, m->nlev - 1, L);
    if (st) return st;
    *bytes = L.total;
    return FEM_OK;
}

fem_status fem_solver_create(const fem_mesh* m, const fem_solve_opts* o, void* ws, size_t ws_bytes, fem_solver** out) {
    fem_status st = check_opts(m, o);
    if (st) return st;
    if (!ws || !out) {
        set_error("fem_solver_create: NULL workspace or output");
        return FEM_ERR_INVALID_ARG;
    }
    if (!m->dev) {
        set_error("fem_solver_create: mesh not uploaded");
        return FEM_ERR_STATE;
    }
    if (((uintptr_t)ws & 255) != 0) {
        set_error("fem_solver_create: workspace not 256-byte aligned");
        return FEM_ERR_INVALID_ARG;
    }
    fem_solver* S = new fem_solver();
    st = S->init(m, *o, m->nlev - 1, (char*)ws, ws_bytes);
    if (st) {
        delete S;
        return st;
    }
    *out = S;
    return FEM_OK;
}

void fem_solver_destroy(fem_solver* S) { delete S; }

fem_status fem_solver_setup(fem_solver* S, const double* k, void* stream) {
    if (!S) {
        set_error("fem_solver_setup: NULL solver");
        return FEM_ERR_INVALID_ARG;
    }
    S->s = (hipStream_t)stream;
    S->ready = false;
    return S->setup(k);
}

fem_status fem_solver_vcycle(fem_solver* S, const double* r, double* z, void* stream) {
    if (!S || !r || !z || r == z) {
        set_error("fem_solver_vcycle: bad arguments");
        return FEM_ERR_INVALID_ARG;
    }
    if (!S->ready) {
        set_error("fem_solver_vcycle: solver not set up");
        return FEM_ERR_STATE;
    }
    S->s = (hipStream_t)stream;
    const bool t = S->timing;
    S->timing = false;
    const fem_status st = S->precondition(r, z);
    S->timing = t;
    if (st) return st;
    return check_launch("fem_solver_vcycle");
}

fem_status fem_solver_solve(fem_solver* S, const double* b, double* x, fem_solve_stats* stats, void* stream) {
    if (!S || !b || !x || b == x) {
        set_error("fem_solver_solve: bad arguments");
        return FEM_ERR_INVALID_ARG;
    }
    if (!S->ready) {
        set_error("fem_solver_solve: solver not set up");
        return FEM_ERR_STATE;
    }
    S->s = (hipStream_t)stream;
    const double t0 = now_ms();
    S->coarse_ms = 0.0;
    S->coarse_iters = 0;
    std::fill(S->level_ms.begin(), S->level_ms.end(), 0.0);
    int it = 0;
    double rel_true = 0.0;
    bool conv = false;
    const fem_status st = S->cg(b, x, it, rel_true, conv);
    if (st) return st;
    const hipError_t e = hipStreamSynchronize(S->s);
    if (e != hipSuccess) {
        set_error(std::string("fem_solver_solve: ") + hipGetErrorString(e));
        return FEM_ERR_HIP;
    }
    const double t1 = now_ms();
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->iterations = it;
        stats->coarse_iterations = S->coarse_iters;
        stats->rel_residual_true = rel_true;
        stats->solve_ms = t1 - t0;
        stats->coarse_ms = S->coarse_ms;
        for (int l = 0; l < S->m->nlev && l < 8; ++l) {
            stats->level_ms[l] = S->level_ms[l];
            stats->lambda_max[l] = S->lmax.size() > (size_t)l ? S->lmax[l] : 0.0;
        }
    }
    if (!conv) {
        set_error("fem_solver_solve: max_it reached before rtol (relative residual " + std::to_string(rel_true) + ")");
        return FEM_WARN_NOT_CONVERGED;
    }
    return FEM_OK;
}

fem_status fem_solver_fmg(fem_solver* S, const double* b, double* x, fem_solve_stats* stats, void* stream) {
    if (!S || !b || !x || b == x) {
        set_error("fem_solver_fmg: bad arguments");
        return FEM_ERR_INVALID_ARG;
    }
    if (!S->ready) {
        set_error("fem_solver_fmg: solver not set up");
        return FEM_ERR_STATE;
    }
    if (S->o.preconditioner != FEM_PC_MG) {
        set_error("fem_solver_fmg: needs the multigrid preconditioner");
        return FEM_ERR_UNSUPPORTED;
    }
    S->s = (hipStream_t)stream;
    S->coarse_iters = 0;
    const bool t = S->timing;
    S->timing = false;
    const double t0 = now_ms();
    double rel = 0.0;
    fem_status st = S->fmg(b, x, rel);
    S->timing = t;
    if (st) return st;
    const hipError_t e = hipStreamSynchronize(S->s);
    if (e != hipSuccess) {
        set_error(std::string("fem_solver_fmg: ") + hipGetErrorString(e));
        return FEM_ERR_HIP;
    }
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->iterations = 1;
        stats->coarse_iterations = S->coarse_iters;
        stats->rel_residual_true = rel;
        stats->solve_ms = now_ms() - t0;
        for (int l = 0; l < S->m->nlev && l < 8; ++l)
            stats->lambda_max[l] = S->lmax.size() > (size_t)l ? S->lmax[l] : 0.0;
    }
    return FEM_OK;
}

fem_status fem_solver_set_level_timing(fem_solver* S, int32_t on) {
    if (!S) {
        set_error("fem_solver_set_level_timing: NULL solver");
        return FEM_ERR_INVALID_ARG;
    }
    S->timing = on != 0;
    return FEM_OK;
}

fem_status fem_mg_cg_solve(const fem_mesh* m, const double* k, const double* b, double* x, const fem_solve_opts* o,
                           void* ws, size_t ws_bytes, fem_solve_stats* stats, void* stream) {
    fem_solver* S = nullptr;
    fem_status st = fem_solver_create(m, o, ws, ws_bytes, &S);
    if (st) return st;
    const double t0 = now_ms();
    st = fem_solver_setup(S, k, stream);
    const double t1 = now_ms();
    if (st == FEM_OK) {
        st = fem_solver_solve(S, b, x, stats, stream);
        if (stats) stats->setup_ms = t1 - t0;
    }
    fem_solver_destroy(S);
    return st;
}

}  // extern "C"
