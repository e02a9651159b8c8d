// Reference tetrahedron for Lagrange P1-P3: basis, gradients, quadrature rules and mass matrix.
// Host code; the results are uploaded as tables that the kernels read with uniform (scalar)
// loads.
//
// Element: continuous Lagrange elements of degree p on the reference tetrahedron with vertices
// (0,0,0), (1,0,0), (0,1,0), (0,0,1) (paper Section 2, Listing 1: FunctionSpace "CG").  Nodes are
// the barycentric multi-indices m, |m| = p, in this local order: vertices; edge nodes, edges
// (0,1),(0,2),(0,3),(1,2),(1,3),(2,3), each from its first vertex towards its second; face nodes,
// faces (0,1,2),(0,1,3),(0,2,3),(1,2,3).  The basis function of node m is the product over the
// four barycentric coordinates l_i of prod_{s < m_i} (p l_i - s) / (s + 1), which is one at its
// node and zero at every other node.
#include "internal.hpp"

#include <cmath>
#include <stdexcept>

namespace fem {

static const int kEdges[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
static const int kFaces[4][3] = {{0, 1, 2}, {0, 1, 3}, {0, 2, 3}, {1, 2, 3}};

void node_multi_indices(int p, std::vector<std::array<int, 4>>& out) {
    out.clear();
    for (int v = 0; v < 4; ++v) {
        std::array<int, 4> m{0, 0, 0, 0};
        m[v] = p;
        out.push_back(m);
    }
    for (auto& e : kEdges)
        for (int s = 1; s < p; ++s) {
            std::array<int, 4> m{0, 0, 0, 0};
            m[e[0]] = p - s;
            m[e[1]] = s;
            out.push_back(m);
        }
    if (p == 3)
        for (auto& f : kFaces) {
            std::array<int, 4> m{0, 0, 0, 0};
            m[f[0]] = m[f[1]] = m[f[2]] = 1;
            out.push_back(m);
        }
}

// One-dimensional factor f_m(t) = prod_{s<m} (p t - s)/(s+1) and its derivative.
static void factor(int p, int m, double t, double& f, double& df) {
    f = 1.0;
    df = 0.0;
    for (int s = 0; s < m; ++s) {
        const double a = (p * t - s) / (s + 1.0), da = p / (s + 1.0);
        df = df * a + f * da;
        f *= a;
    }
}

void eval_basis_grad(int p, const double xi[3], double* phi, double* dphi) {
    std::vector<std::array<int, 4>> mi;
    node_multi_indices(p, mi);
    const double lam[4] = {1.0 - xi[0] - xi[1] - xi[2], xi[0], xi[1], xi[2]};
    // d lambda_i / d xi_d
    const double dl[4][3] = {{-1, -1, -1}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    for (size_t n = 0; n < mi.size(); ++n) {
        double f[4], df[4];
        for (int i = 0; i < 4; ++i) factor(p, mi[n][i], lam[i], f[i], df[i]);
        if (phi) phi[n] = f[0] * f[1] * f[2] * f[3];
        if (dphi)
            for (int d = 0; d < 3; ++d) {
                double g = 0.0;
                for (int i = 0; i < 4; ++i) {
                    double prod = df[i];
                    for (int j = 0; j < 4; ++j)
                        if (j != i) prod *= f[j];
                    g += prod * dl[i][d];
                }
                dphi[n * 3 + d] = g;
            }
    }
}

// ---- polynomials in (x, y, z) with double coefficients, total degree <= 6 ----
namespace {
constexpr int PD = 7;
struct Poly {
    double c[PD][PD][PD] = {};
};
Poly mul(const Poly& a, const Poly& b) {
    Poly r;
    for (int i = 0; i < PD; ++i)
        for (int j = 0; i + j < PD; ++j)
            for (int k = 0; i + j + k < PD; ++k) {
                if (a.c[i][j][k] == 0.0) continue;
                for (int u = 0; i + u < PD; ++u)
                    for (int v = 0; j + v < PD && i + j + u + v < PD; ++v)
                        for (int w = 0; k + w < PD && i + j + k + u + v + w < PD; ++w)
                            r.c[i + u][j + v][k + w] += a.c[i][j][k] * b.c[u][v][w];
            }
    return r;
}
double fact(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}
// int over the reference tetrahedron of x^a y^b z^c = a! b! c! / (a+b+c+3)!
double mono_int(int a, int b, int c) { return fact(a) * fact(b) * fact(c) / fact(a + b + c + 3); }
double integrate(const Poly& p) {
    double s = 0.0;
    for (int i = 0; i < PD; ++i)
        for (int j = 0; i + j < PD; ++j)
            for (int k = 0; i + j + k < PD; ++k) s += p.c[i][j][k] * mono_int(i, j, k);
    return s;
}
Poly lambda_poly(int i) {
    Poly r;
    if (i == 0) {
        r.c[0][0][0] = 1.0;
        r.c[1][0][0] = r.c[0][1][0] = r.c[0][0][1] = -1.0;
    } else if (i == 1) {
        r.c[1][0][0] = 1.0;
    } else if (i == 2) {
        r.c[0][1][0] = 1.0;
    } else {
        r.c[0][0][1] = 1.0;
    }
    return r;
}
Poly basis_poly(int p, const std::array<int, 4>& m) {
    Poly r;
    r.c[0][0][0] = 1.0;
    for (int i = 0; i < 4; ++i)
        for (int s = 0; s < m[i]; ++s) {
            Poly f = lambda_poly(i);
            for (int a = 0; a < PD; ++a)
                for (int b = 0; b < PD; ++b)
                    for (int c = 0; c < PD; ++c) f.c[a][b][c] *= p / (s + 1.0);
            f.c[0][0][0] -= s / (s + 1.0);
            r = mul(r, f);
        }
    return r;
}
}  // namespace

void mass_matrix(int p, std::vector<double>& M) {
    std::vector<std::array<int, 4>> mi;
    node_multi_indices(p, mi);
    const int n = (int)mi.size();
    std::vector<Poly> b(n);
    for (int i = 0; i < n; ++i) b[i] = basis_poly(p, mi[i]);
    M.assign(n * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) M[i * n + j] = integrate(mul(b[i], b[j]));
}

// ---- quadrature rules ----
// Symmetric rules on the reference tetrahedron (weights sum to 1/6), given by orbits of
// barycentric points.  Orbit S4: centroid.  S31(a): the 4 points with barycentric (a,a,a,1-3a)
// permuted.  S22(a): the 6 points (a,a,1/2-a,1/2-a) permuted.
//   degree 1:  S4 (w = 1/6)
//   degree 2:  S31(a), a = (5 - sqrt 5)/20, w = 1/24                      (Hammer-Stroud)
//   degree 3:  S4 (w = -2/15), S31(1/6) (w = 3/40)                       (Hammer-Stroud)
//   degree 4:  S4 (w = -74/5625), S31(1/14) (w = 343/45000),
//              S22((1 - sqrt(5/14))/4) (w = 56/2250)                      (Keast)
//   degree 5:  S31(a1), S31(a2), S22(b), 14 points (Walkington); the orbit parameters and
//              weights are refined below by Gauss-Newton on the moment equations.
// Every rule is checked at start-up to integrate all monomials up to its degree to 2e-15
// relative; a failure throws.
namespace {
struct Orbit {
    int kind;  // 0: S4, 1: S31, 2: S22
    double a, w;
};
void expand(const std::vector<Orbit>& orbits, Rule& r) {
    r.x.clear();
    r.w.clear();
    r.lam.clear();
    auto push = [&](double l0, double l1, double l2, double l3, double w) {
        r.lam.insert(r.lam.end(), {l0, l1, l2, l3});
        r.x.insert(r.x.end(), {l1, l2, l3});
        r.w.push_back(w);
    };
    for (auto& o : orbits) {
        if (o.kind == 0) {
            push(0.25, 0.25, 0.25, 0.25, o.w);
        } else if (o.kind == 1) {
            const double a = o.a, b = 1.0 - 3.0 * o.a;
            push(b, a, a, a, o.w);
            push(a, b, a, a, o.w);
            push(a, a, b, a, o.w);
            push(a, a, a, b, o.w);
        } else {
            const double a = o.a, b = 0.5 - o.a;
            const int pairs[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
            for (auto& pr : pairs) {
                double l[4] = {b, b, b, b};
                l[pr[0]] = a;
                l[pr[1]] = a;
                push(l[0], l[1], l[2], l[3], o.w);
            }
        }
    }
}
double moment_error(const Rule& r, int degree, std::vector<double>* resid) {
    double worst = 0.0;
    if (resid) resid->clear();
    for (int a = 0; a <= degree; ++a)
        for (int b = 0; a + b <= degree; ++b)
            for (int c = 0; a + b + c <= degree; ++c) {
                double s = 0.0;
                for (size_t q = 0; q < r.w.size(); ++q)
                    s += r.w[q] * std::pow(r.x[3 * q], a) * std::pow(r.x[3 * q + 1], b) *
                         std::pow(r.x[3 * q + 2], c);
                const double ex = mono_int(a, b, c);
                if (resid) resid->push_back((s - ex) / ex);
                worst = std::max(worst, std::fabs(s - ex) / ex);
            }
    return worst;
}
// Gauss-Newton on the orbit parameters (a, w) of all orbits.
void refine(std::vector<Orbit>& orbits, int degree) {
    Rule r;
    for (int it = 0; it < 20; ++it) {
        expand(orbits, r);
        std::vector<double> f0;
        if (moment_error(r, degree, &f0) < 1e-16) return;
        std::vector<double*> params;
        for (auto& o : orbits) {
            if (o.kind != 0) params.push_back(&o.a);
            params.push_back(&o.w);
        }
        const int np = (int)params.size(), ne = (int)f0.size();
        std::vector<double> J(ne * np);
        for (int j = 0; j < np; ++j) {
            const double save = *params[j], h = 1e-7 * std::max(1e-3, std::fabs(save));
            *params[j] = save + h;
            expand(orbits, r);
            std::vector<double> f1;
            moment_error(r, degree, &f1);
            *params[j] = save;
            for (int i = 0; i < ne; ++i) J[i * np + j] = (f1[i] - f0[i]) / h;
        }
        // normal equations (J^T J) d = -J^T f
        std::vector<double> A(np * np, 0.0), g(np, 0.0);
        for (int i = 0; i < ne; ++i)
            for (int j = 0; j < np; ++j) {
                g[j] -= J[i * np + j] * f0[i];
                for (int k = 0; k < np; ++k) A[j * np + k] += J[i * np + j] * J[i * np + k];
            }
        for (int c = 0; c < np; ++c) {  // Gaussian elimination with partial pivoting
            int piv = c;
            for (int rr = c + 1; rr < np; ++rr)
                if (std::fabs(A[rr * np + c]) > std::fabs(A[piv * np + c])) piv = rr;
            for (int k = 0; k < np; ++k) std::swap(A[c * np + k], A[piv * np + k]);
            std::swap(g[c], g[piv]);
            for (int rr = c + 1; rr < np; ++rr) {
                const double f = A[rr * np + c] / A[c * np + c];
                for (int k = c; k < np; ++k) A[rr * np + k] -= f * A[c * np + k];
                g[rr] -= f * g[c];
            }
        }
        std::vector<double> d(np);
        for (int c = np - 1; c >= 0; --c) {
            double s = g[c];
            for (int k = c + 1; k < np; ++k) s -= A[c * np + k] * d[k];
            d[c] = s / A[c * np + c];
        }
        for (int j = 0; j < np; ++j) *params[j] += d[j];
    }
}
Rule make_rule(int degree) {
    std::vector<Orbit> o;
    if (degree <= 1) {
        o = {{0, 0.0, 1.0 / 6.0}};
    } else if (degree == 2) {
        o = {{1, (5.0 - std::sqrt(5.0)) / 20.0, 1.0 / 24.0}};
    } else if (degree == 3) {
        o = {{0, 0.0, -2.0 / 15.0}, {1, 1.0 / 6.0, 3.0 / 40.0}};
    } else if (degree == 4) {
        o = {{0, 0.0, -74.0 / 5625.0}, {1, 1.0 / 14.0, 343.0 / 45000.0},
             {2, (1.0 - std::sqrt(5.0 / 14.0)) / 4.0, 56.0 / 2250.0}};
    } else if (degree == 5) {
        o = {{1, 0.0927352503108912, 0.01224884051939366},
             {1, 0.3108859192633006, 0.01878132095300264},
             {2, 0.0455037041256496, 0.007091003462846911}};
        refine(o, 5);
    } else {
        throw std::invalid_argument("no quadrature rule of that degree");
    }
    Rule r;
    expand(o, r);
    r.degree = degree;
    const double err = moment_error(r, std::max(degree, 0), nullptr);
    if (err > 2e-15) throw std::runtime_error("quadrature rule failed its exactness check");
    return r;
}
}  // namespace

const Rule& rule_for_degree(int degree) {
    static Rule rules[6];
    static bool made[6] = {false, false, false, false, false, false};
    if (degree < 1) degree = 1;
    if (degree > 5) throw std::invalid_argument("quadrature degree > 5");
    if (!made[degree]) {
        rules[degree] = make_rule(degree);
        made[degree] = true;
    }
    return rules[degree];
}

double rule_exactness_error(int degree) {
    const Rule& r = rule_for_degree(degree);
    return moment_error(r, degree, nullptr);
}

}  // namespace fem
