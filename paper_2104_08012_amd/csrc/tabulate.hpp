// Compile-time quadrature tabulations for the stiffness kernels.
//
// The element integral int_K k grad(u).grad(v) is evaluated with a symmetric quadrature rule that
// is exact for the integrand (degree 2p-2 for k = 1, 2p-1 for a P1 coefficient):
//   P1:            the centroid, weight 1/6;
//   P2, k = 1:     S31(a) with a = (5 - sqrt 5)/20, weights 1/24 (degree 2);
//   P2, P1 k:      centroid (weight -2/15) and S31(1/6) (weights 3/40) (degree 3);
//   P3, k = 1:     centroid (-74/5625), S31(1/14) (343/45000), S22((1 - sqrt(5/14))/4) (56/2250)
//                  (degree 4, 11 points);
//   P3, P1 k:      S31(a1), S31(a2), S22(b), 14 points (degree 5), parameters to double precision.
// The reference gradients of the Lagrange basis at the points are computed here by constexpr
// evaluation of the product form of the basis (phi_m = prod_i prod_{s<m_i} (p l_i - s)/(s+1)),
// so the kernels see them as literals and drop the zero entries.  The host builds the same rules
// independently (refelem.cpp) and checks their exactness; tests/tab_check.cpp compares the two.
#pragma once
#include "common.hpp"

namespace fem {

template <int P>
struct NodeList {
    static constexpr int NL = nloc_of(P);
    int m[NL][4];
    constexpr NodeList() : m{} {
        int n = 0;
        for (int v = 0; v < 4; ++v) {
            for (int k = 0; k < 4; ++k) m[n][k] = (k == v) ? P : 0;
            ++n;
        }
        const int ea[6] = {0, 0, 0, 1, 1, 2}, eb[6] = {1, 2, 3, 2, 3, 3};
        for (int e = 0; e < 6; ++e)
            for (int s = 1; s < P; ++s) {
                for (int k = 0; k < 4; ++k) m[n][k] = 0;
                m[n][ea[e]] = P - s;
                m[n][eb[e]] = s;
                ++n;
            }
        const int fa[4] = {0, 0, 0, 1}, fb[4] = {1, 1, 2, 2}, fc[4] = {2, 3, 3, 3};
        if (P == 3)
            for (int f = 0; f < 4; ++f) {
                for (int k = 0; k < 4; ++k) m[n][k] = 0;
                m[n][fa[f]] = m[n][fb[f]] = m[n][fc[f]] = 1;
                ++n;
            }
    }
};

template <int P, bool KVAR>
struct StiffTab {
    static constexpr int NL = nloc_of(P), NQ = nq_of(P, KVAR);
    double w[NQ];
    double lam[NQ][4];
    double D[NQ][3][NL];   // reference gradient d phi_i / d xi_d at point q

    constexpr StiffTab() : w{}, lam{}, D{} {
        // points (barycentric) and weights
        if (P == 1) {
            set_point(0, 0.25, 0.25, 0.25, 0.25, 1.0 / 6.0);
        } else if (P == 3 && !KVAR) {
            set_point(0, 0.25, 0.25, 0.25, 0.25, -74.0 / 5625.0);
            int q = 1;
            q = s31(q, 1.0 / 14.0, 343.0 / 45000.0);
            s22(q, 0.1005964238332008, 56.0 / 2250.0);
        } else if (P == 3) {
            int q = 0;
            q = s31(q, 0.092735250310891248, 0.012248840519393664);
            q = s31(q, 0.31088591926330061, 0.018781320953002674);
            s22(q, 0.045503704125649434, 0.0070910034628468826);
        } else if (!KVAR) {
            const double a = 0.13819660112501050975, b = 0.58541019662496847076;  // (5 -+ sqrt5)/20 ..
            set_point(0, b, a, a, a, 1.0 / 24.0);
            set_point(1, a, b, a, a, 1.0 / 24.0);
            set_point(2, a, a, b, a, 1.0 / 24.0);
            set_point(3, a, a, a, b, 1.0 / 24.0);
        } else {
            set_point(0, 0.25, 0.25, 0.25, 0.25, -2.0 / 15.0);
            const double a = 1.0 / 6.0, b = 0.5;
            set_point(1, b, a, a, a, 3.0 / 40.0);
            set_point(2, a, b, a, a, 3.0 / 40.0);
            set_point(3, a, a, b, a, 3.0 / 40.0);
            set_point(4, a, a, a, b, 3.0 / 40.0);
        }
        const NodeList<P> nodes{};
        const double dl[4][3] = {{-1, -1, -1}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
        for (int q = 0; q < NQ; ++q)
            for (int i = 0; i < NL; ++i) {
                double f[4] = {1, 1, 1, 1}, df[4] = {0, 0, 0, 0};
                for (int k = 0; k < 4; ++k)
                    for (int s = 0; s < nodes.m[i][k]; ++s) {
                        const double a = (P * lam[q][k] - s) / (s + 1.0), da = P / (s + 1.0);
                        df[k] = df[k] * a + f[k] * da;
                        f[k] *= a;
                    }
                for (int d = 0; d < 3; ++d) {
                    double g = 0.0;
                    for (int k = 0; k < 4; ++k) {
                        double prod = df[k];
                        for (int j = 0; j < 4; ++j)
                            if (j != k) prod *= f[j];
                        g += prod * dl[k][d];
                    }
                    D[q][d][i] = g;
                }
            }
    }
    // the 4 points (b,a,a,a) permuted, b = 1 - 3a
    constexpr int s31(int q, double a, double wt) {
        const double b = 1.0 - 3.0 * a;
        set_point(q, b, a, a, a, wt);
        set_point(q + 1, a, b, a, a, wt);
        set_point(q + 2, a, a, b, a, wt);
        set_point(q + 3, a, a, a, b, wt);
        return q + 4;
    }
    // the 6 points with a at the coordinate pairs (0,1),(0,2),(0,3),(1,2),(1,3),(2,3), b = 1/2 - a
    constexpr int s22(int q, double a, double wt) {
        const double b = 0.5 - a;
        const int pr[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
        for (int k = 0; k < 6; ++k) {
            double l[4] = {b, b, b, b};
            l[pr[k][0]] = a;
            l[pr[k][1]] = a;
            set_point(q + k, l[0], l[1], l[2], l[3], wt);
        }
        return q + 6;
    }
    constexpr void set_point(int q, double l0, double l1, double l2, double l3, double wt) {
        lam[q][0] = l0;
        lam[q][1] = l1;
        lam[q][2] = l2;
        lam[q][3] = l3;
        w[q] = wt;
    }
};

// Reference gradients of the basis at the four vertices, D[v][d][i] = d phi_i / d xi_d at vertex v.
// With k = 1 and an affine cell, grad u is linear for P2 (degree p - 1 in general), so
// int_K G grad(u) . grad(phi_j) = sum_v,v' M1[v][v'] (G g_v) . D[v'][.][j] with g_v the reference
// gradient at vertex v and M1 the reference P1 mass matrix (1 + delta_vv') / 120: exact, and sparser
// than interior quadrature because most basis gradients vanish at the vertices.
template <int P>
struct VertexGrad {
    static constexpr int NL = nloc_of(P);
    double D[4][3][NL];
    constexpr VertexGrad() : D{} {
        const NodeList<P> nodes{};
        const double dl[4][3] = {{-1, -1, -1}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
        for (int v = 0; v < 4; ++v)
            for (int i = 0; i < NL; ++i) {
                double lam[4] = {0, 0, 0, 0};
                lam[v] = 1.0;
                double f[4] = {1, 1, 1, 1}, df[4] = {0, 0, 0, 0};
                for (int k = 0; k < 4; ++k)
                    for (int s = 0; s < nodes.m[i][k]; ++s) {
                        const double a = (P * lam[k] - s) / (s + 1.0), da = P / (s + 1.0);
                        df[k] = df[k] * a + f[k] * da;
                        f[k] *= a;
                    }
                for (int d = 0; d < 3; ++d) {
                    double g = 0.0;
                    for (int k = 0; k < 4; ++k) {
                        double prod = df[k];
                        for (int j = 0; j < 4; ++j)
                            if (j != k) prod *= f[j];
                        g += prod * dl[k][d];
                    }
                    D[v][d][i] = g;
                }
            }
    }
};

// Local node i of the path tetrahedron t sits at cube-lattice point (pa, pb, pc) in [0, P]^3.
template <int P>
struct CubeNodes {
    static constexpr int NL = nloc_of(P), PC = P + 1, NCP = PC * PC * PC;
    int cp[6][NL];        // tetrahedron t, node i -> cube point index
    constexpr CubeNodes() : cp{} {
        const NodeList<P> nodes{};
        for (int t = 0; t < 6; ++t) {
            const int s0 = perm_axis(t, 0), s1 = perm_axis(t, 1);
            int V[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {1, 1, 1}};
            V[1][s0] = 1;
            V[2][s0] = 1;
            V[2][s1] = 1;
            for (int i = 0; i < NL; ++i) {
                int X[3] = {0, 0, 0};
                for (int v = 0; v < 4; ++v)
                    for (int k = 0; k < 3; ++k) X[k] += nodes.m[i][v] * V[v][k];
                const int j = X[0] + PC * (X[1] + PC * X[2]);
                cp[t][i] = j;
            }
        }
    }
};

}  // namespace fem
