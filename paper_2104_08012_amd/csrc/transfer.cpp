// Tables of the lattice transfer kernels (host, built once per mesh).
//
// Uniform refinement halves the lattice spacing: the fine P_p dofs of a coarse cube sit at the
// points r / (2p) of the cube, r in [0, 2p]^3 (in units of the coarse cube).  Prolongation
// interpolates the coarse function there (Section 4: nested spaces, the coarse correction is
// carried to the finer level), so each fine dof takes sum_i phi_i(lambda) x_c[node i] over the
// nodes of the coarse tetrahedron holding the point.
//  * Prolongation table: for every local position r, the nodes of that tetrahedron (offsets in
//    [0, p]^3 from the cube's first coarse node) with nonzero weights phi_i(lambda), padded with
//    zero weights to nloc entries.  The tetrahedron is the path tetrahedron whose axis order sorts
//    r decreasingly, with lambda = (2p - r_s0, r_s0 - r_s1, r_s1 - r_s2, r_s2) / (2p); on a face
//    shared by several tetrahedra every choice gives the same values (continuity).  The basis
//    values are products of (k - 2s) / (2 (s + 1)) factors: computed as exact integer ratios and
//    rounded once, so weights at coinciding nodes are exactly 1 and 0.
//  * Restriction stencils (R = P^T): the coarse node J gathers sum_f P[f][J] r_f over the fine
//    points f = 2 J + d, d in [-2p, 2p]^3 (the support of its basis function).  P[f][J] depends
//    only on d and on the residue class of J modulo p, so one list of (d, weight) per class,
//    read from the prolongation table at an interior representative of the class, serves every
//    coarse node; points outside the fine lattice are skipped by the kernel.
#include <array>
#include <cmath>
#include <cstdint>
#include <stdexcept>
#include <vector>

#include "internal.hpp"

namespace fem {

namespace {

void path_vertices(int t, int V[4][3]) {
    for (int w = 0; w < 4; ++w)
        for (int d = 0; d < 3; ++d) V[w][d] = 0;
    V[1][perm_axis(t, 0)] = 1;
    V[2][perm_axis(t, 0)] = 1;
    V[2][perm_axis(t, 1)] = 1;
    V[3][0] = V[3][1] = V[3][2] = 1;
}

// Local cube offset of node i of path tetrahedron t, packed a0 | a1 << 8 | a2 << 16.
int node_offset(const std::array<int, 4>& m, const int V[4][3]) {
    int a[3] = {0, 0, 0};
    for (int w = 0; w < 4; ++w)
        for (int d = 0; d < 3; ++d) a[d] += m[w] * V[w][d];
    return a[0] | (a[1] << 8) | (a[2] << 16);
}

}  // namespace

void build_transfer_tables(fem_mesh& m) {
    const int p = m.p, S = 2 * p + 1, NPOS = S * S * S, nl = nloc_of(p);
    std::vector<std::array<int, 4>> mi;
    node_multi_indices(p, mi);
    m.pt_ne = nl;
    m.pt_off.assign((size_t)NPOS * nl, 0);
    m.pt_w64.assign((size_t)NPOS * nl, 0.0);
    for (int rz = 0; rz < S; ++rz)
        for (int ry = 0; ry < S; ++ry)
            for (int rx = 0; rx < S; ++rx) {
                const int r[3] = {rx, ry, rz}, pos = rx + S * (ry + S * rz);
                int t = -1;
                for (int tt = 0; tt < 6 && t < 0; ++tt)
                    if (r[perm_axis(tt, 0)] >= r[perm_axis(tt, 1)] && r[perm_axis(tt, 1)] >= r[perm_axis(tt, 2)]) t = tt;
                const int s0 = perm_axis(t, 0), s1 = perm_axis(t, 1), s2 = perm_axis(t, 2);
                // 2p lambda: integers
                const int k[4] = {2 * p - r[s0], r[s0] - r[s1], r[s1] - r[s2], r[s2]};
                int V[4][3];
                path_vertices(t, V);
                int e = 0;
                for (int i = 0; i < nl; ++i) {
                    // phi = prod_w prod_{s < m_w} (p lambda_w - s) / (s + 1), p lambda_w = k_w / 2
                    int64_t num = 1, den = 1;
                    for (int w = 0; w < 4; ++w)
                        for (int s = 0; s < mi[i][w]; ++s) {
                            num *= (k[w] - 2 * s);
                            den *= 2 * (s + 1);
                        }
                    if (num == 0) continue;
                    m.pt_off[(size_t)pos * nl + e] = node_offset(mi[i], V);
                    m.pt_w64[(size_t)pos * nl + e] = (double)num / (double)den;
                    ++e;
                }
                // the weights are a partition of unity at every point
                double sum = 0.0;
                for (int q = 0; q < e; ++q) sum += m.pt_w64[(size_t)pos * nl + q];
                if (std::abs(sum - 1.0) > 1e-14) throw std::runtime_error("prolongation weights do not sum to 1");
            }
    m.pt_w32.assign(m.pt_w64.begin(), m.pt_w64.end());

    // restriction stencils per residue class of the coarse node
    const int NCL = p * p * p, D = 4 * p + 1;
    m.rs_start.assign(NCL + 1, 0);
    m.rs_off.clear();
    m.rs_w64.clear();
    for (int cls = 0; cls < NCL; ++cls) {
        m.rs_start[cls] = (int32_t)m.rs_off.size();
        const int rho[3] = {cls % p, (cls / p) % p, cls / (p * p)};
        int J[3];
        for (int d = 0; d < 3; ++d) J[d] = rho[d] + 3 * p;   // interior representative
        for (int dz = -2 * p; dz <= 2 * p; ++dz)
            for (int dy = -2 * p; dy <= 2 * p; ++dy)
                for (int dx = -2 * p; dx <= 2 * p; ++dx) {
                    const int F[3] = {2 * J[0] + dx, 2 * J[1] + dy, 2 * J[2] + dz};
                    int c[3], r[3];
                    for (int d = 0; d < 3; ++d) {
                        c[d] = F[d] / (2 * p);
                        r[d] = F[d] - 2 * p * c[d];
                    }
                    const int pos = r[0] + S * (r[1] + S * r[2]);
                    double w = 0.0;
                    for (int e = 0; e < nl; ++e) {
                        const double we = m.pt_w64[(size_t)pos * nl + e];
                        if (we == 0.0) continue;
                        const int o = m.pt_off[(size_t)pos * nl + e];
                        const int a[3] = {o & 255, (o >> 8) & 255, o >> 16};
                        if (p * c[0] + a[0] == J[0] && p * c[1] + a[1] == J[1] && p * c[2] + a[2] == J[2]) w = we;
                    }
                    if (w == 0.0) continue;
                    m.rs_off.push_back((dx + 2 * p) + D * ((dy + 2 * p) + D * (dz + 2 * p)));
                    m.rs_w64.push_back(w);
                }
    }
    m.rs_start[NCL] = (int32_t)m.rs_off.size();
    m.rs_w32.assign(m.rs_w64.begin(), m.rs_w64.end());
    // linear offsets of the stencil points on each fine lattice (interior coarse points need no
    // bounds checks: F = 2 J + d stays inside when every coordinate of J is in [p, L_c - 1 - p])
    for (int l = 0; l + 1 < m.nlev; ++l) {
        const int64_t Lf = m.lev[l + 1].L;
        auto& lin = m.lev[l].rs_lin;
        lin.resize(m.rs_off.size());
        for (size_t e = 0; e < m.rs_off.size(); ++e) {
            const int o = m.rs_off[e];
            const int64_t dx = o % D - 2 * p, dy = (o / D) % D - 2 * p, dz = o / (D * D) - 2 * p;
            lin[e] = (int32_t)(dx + Lf * (dy + Lf * dz));
        }
    }
}

}  // namespace fem
