// Mesh hierarchy on the host: the tetrahedral unit cube of the paper (Section 2, Listing 1:
// UnitCubeMesh(N, N, N), MeshHierarchy(mesh, r)), its P_p numbering, the per-cell geometric
// factors and the tables the kernels use.
//
// Cube split: each cube is cut into the 6 tetrahedra that share its main diagonal; uniform
// refinement (new vertices at edge midpoints) maps the split of n^3 cubes onto the split of
// (2n)^3 cubes, so level l is the split of (n 2^l)^3 cubes with vertices at edge midpoints of
// level l-1 (and only level 0 may be perturbed).
//
// Layout for the kernels:
//  * cells are ordered brick by brick: bricks of B^3 cubes (B = 4, 2 or 1, the largest that
//    divides n), bricks x-fastest; inside a brick the cells are grouped by tetrahedron type t
//    (the axis order of the path), cubes x-fastest within a group:
//    c = brick * 6 B^3 + t * B^3 + cube_local, so that threads handling consecutive cubes read
//    consecutive entries of every per-cell array.
//  * cell-to-dof map: structure of arrays, map[i * C + c] for local node i, int32 with the sign
//    bit set on boundary dofs.
//  * geometric factor G = |det J| J^-1 J^-T: structure of arrays, 6 entries (00,11,22,01,02,12),
//    FP64 and an FP32 copy.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <stdexcept>

#include "internal.hpp"
#include "tabulate.hpp"

namespace fem {

static int choose_brick(int n) { return (n % 4 == 0) ? 4 : (n % 2 == 0) ? 2 : 1; }

static void build_red(RedTable& t, int po, int B) {
    t.po = po;
    t.B = B;
    t.NC = 6 * B * B * B;
    const int PB = po * B, QS = PB + 1;
    t.Q = QS * QS * QS;
    std::vector<std::array<int, 4>> mi;
    node_multi_indices(po, mi);
    const int nl = (int)mi.size();
    std::vector<std::vector<int32_t>> lists(t.Q);
    t.q_of.assign((size_t)t.NC * nl, -1);
    for (int cl = 0; cl < t.NC; ++cl) {
        const int B3 = B * B * B, cube = cl % B3, tt = cl / B3;
        const int lx = cube % B, ly = (cube / B) % B, lz = cube / (B * B);
        int V[4][3];
        V[0][0] = lx; V[0][1] = ly; V[0][2] = lz;
        for (int k = 0; k < 3; ++k) V[1][k] = V[0][k];
        V[1][perm_axis(tt, 0)] += 1;
        for (int k = 0; k < 3; ++k) V[2][k] = V[1][k];
        V[2][perm_axis(tt, 1)] += 1;
        for (int k = 0; k < 3; ++k) V[3][k] = V[0][k] + 1;
        for (int i = 0; i < nl; ++i) {
            int X[3] = {0, 0, 0};
            for (int v = 0; v < 4; ++v)
                for (int k = 0; k < 3; ++k) X[k] += mi[i][v] * V[v][k];
            const int q = X[0] + QS * (X[1] + QS * X[2]);
            lists[q].push_back(i * t.NC + cl);
            t.q_of[(size_t)cl * nl + i] = q;
        }
    }
    t.off.assign(t.Q + 1, 0);
    t.ent.clear();
    t.slot.assign(t.Q, -1);
    int nslot = 0;
    for (int q = 0; q < t.Q; ++q) {
        std::sort(lists[q].begin(), lists[q].end());
        t.off[q] = (int32_t)t.ent.size();
        t.ent.insert(t.ent.end(), lists[q].begin(), lists[q].end());
        const int a = q % QS, b = (q / QS) % QS, c = q / (QS * QS);
        const bool inside = a > 0 && a < PB && b > 0 && b < PB && c > 0 && c < PB;
        if (!inside) t.slot[q] = nslot++;
    }
    t.off[t.Q] = (int32_t)t.ent.size();
    t.QB = nslot;
}

static int find_red(fem_mesh& m, int po, int B) {
    for (size_t i = 0; i < m.red.size(); ++i)
        if (m.red[i].po == po && m.red[i].B == B) return (int)i;
    RedTable t;
    build_red(t, po, B);
    m.red.push_back(std::move(t));
    return (int)m.red.size() - 1;
}

static void cell_vertices(const HostLevel& L, int64_t c, int V[4][3]) {
    const int64_t brick = c / L.NC;
    const int cl = (int)(c % L.NC);
    const int B = L.B, B3 = B * B * B;
    const int cube = cl % B3, t = cl / B3;
    const int bx = (int)(brick % L.nb), by = (int)((brick / L.nb) % L.nb), bz = (int)(brick / ((int64_t)L.nb * L.nb));
    V[0][0] = bx * B + cube % B;
    V[0][1] = by * B + (cube / B) % B;
    V[0][2] = bz * B + cube / (B * B);
    for (int k = 0; k < 3; ++k) V[1][k] = V[0][k];
    V[1][perm_axis(t, 0)] += 1;
    for (int k = 0; k < 3; ++k) V[2][k] = V[1][k];
    V[2][perm_axis(t, 1)] += 1;
    for (int k = 0; k < 3; ++k) V[3][k] = V[0][k] + 1;
}

// G = adj(M) adj(M)^T / |det M| (= |det M| M^-1 M^-T) for M with the edge vectors as columns;
// returns det M.
static double geometric_factor(const double M[3][3], double g6[6]) {
    double adj[3][3];
    adj[0][0] = M[1][1] * M[2][2] - M[1][2] * M[2][1];
    adj[0][1] = M[0][2] * M[2][1] - M[0][1] * M[2][2];
    adj[0][2] = M[0][1] * M[1][2] - M[0][2] * M[1][1];
    adj[1][0] = M[1][2] * M[2][0] - M[1][0] * M[2][2];
    adj[1][1] = M[0][0] * M[2][2] - M[0][2] * M[2][0];
    adj[1][2] = M[0][2] * M[1][0] - M[0][0] * M[1][2];
    adj[2][0] = M[1][0] * M[2][1] - M[1][1] * M[2][0];
    adj[2][1] = M[0][1] * M[2][0] - M[0][0] * M[2][1];
    adj[2][2] = M[0][0] * M[1][1] - M[0][1] * M[1][0];
    const double det = M[0][0] * adj[0][0] + M[0][1] * adj[1][0] + M[0][2] * adj[2][0];
    double G[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += adj[a][k] * adj[b][k];
            G[a][b] = s / std::fabs(det);
        }
    g6[0] = G[0][0];
    g6[1] = G[1][1];
    g6[2] = G[2][2];
    g6[3] = G[0][1];
    g6[4] = G[0][2];
    g6[5] = G[1][2];
    return det;
}

static void build_level(HostLevel& L, const std::vector<std::array<int, 4>>& mi) {
    const int n = L.n, p = L.p, nl = L.nloc;
    L.B = choose_brick(n);
    L.nb = n / L.B;
    L.NC = 6 * L.B * L.B * L.B;
    L.L = p * n + 1;
    L.C = 6LL * n * n * n;
    L.N = (int64_t)L.L * L.L * L.L;
    // the kernels address every array (and every structure-of-arrays plane) with 32-bit byte
    // offsets of 8-byte entries
    if (L.C >= (1LL << 29) || L.N >= (1LL << 29))
        throw std::runtime_error("level too large: at most 2^29 cells and 2^29 dofs per level");
    L.NI = (int64_t)(L.L - 2) * (L.L - 2) * (L.L - 2);
    L.NV = (int64_t)(n + 1) * (n + 1) * (n + 1);
    L.nbricks = (int64_t)L.nb * L.nb * L.nb;
    const int64_t C = L.C;
    L.map.assign((size_t)nl * C, 0);
    L.G64.assign((size_t)6 * C, 0.0);
    L.G32.assign((size_t)6 * C, 0.0f);
    const int N1 = n + 1, Lp = L.L;
    for (int64_t c = 0; c < C; ++c) {
        int V[4][3];
        cell_vertices(L, c, V);
        for (int i = 0; i < nl; ++i) {
            int X[3] = {0, 0, 0};
            for (int v = 0; v < 4; ++v)
                for (int k = 0; k < 3; ++k) X[k] += mi[i][v] * V[v][k];
            const bool bnd = X[0] == 0 || X[1] == 0 || X[2] == 0 || X[0] == Lp - 1 || X[1] == Lp - 1 ||
                             X[2] == Lp - 1;
            const int64_t g = X[0] + (int64_t)Lp * (X[1] + (int64_t)Lp * X[2]);
            L.map[(size_t)i * C + c] = (int32_t)((uint32_t)g | (bnd ? kBoundaryBit : 0u));
        }
        double x[4][3];
        for (int v = 0; v < 4; ++v) {
            const int64_t vid = V[v][0] + (int64_t)N1 * (V[v][1] + (int64_t)N1 * V[v][2]);
            for (int k = 0; k < 3; ++k) x[v][k] = L.vxyz[3 * vid + k];
        }
        double J[3][3];  // columns are the edges x1-x0, x2-x0, x3-x0
        for (int r = 0; r < 3; ++r)
            for (int col = 0; col < 3; ++col) J[r][col] = x[col + 1][r] - x[0][r];
        double g6[6];
        const double det = geometric_factor(J, g6);
        for (int e = 0; e < 6; ++e) {
            L.G64[(size_t)e * C + c] = g6[e];
            L.G32[(size_t)e * C + c] = (float)g6[e];
        }
        // orientation of the path tetrahedron on the uniform lattice: sign of the permutation
        const int t = (int)((c % L.NC) / ((int64_t)L.B * L.B * L.B));
        const double sgn = (t == 0 || t == 3 || t == 4) ? 1.0 : -1.0;
        const double h = 1.0 / n;
        if (!(det * sgn > 0.05 * h * h * h)) {
            throw std::runtime_error("mesh cell inverted or degenerate (jitter too large)");
        }
    }
}

// Cube-kernel data: the vertex coordinates in structure-of-arrays order.  The kernel addresses dofs
// by their lattice point, the numbering validate_level checks for every map entry.
static void build_cube_data(HostLevel& L) {
    const int64_t NV = L.NV;
    L.vsoa.assign((size_t)3 * NV, 0.0);
    for (int64_t v = 0; v < NV; ++v)
        for (int a = 0; a < 3; ++a) L.vsoa[(size_t)a * NV + v] = L.vxyz[(size_t)3 * v + a];
    L.cube = true;
}

// Geometric factors of every level from the coarsest level's cells (see fem_mesh::geo).  The
// coarsest cell (cube q0, type t0) has lattice edges E_t0 (integer, det +-1) and physical edges
// J0, so its lattice-to-physical map is L = J0 E_t0^-1; a type-t tetrahedron of the same lattice
// scale inside it has physical edges L E_t.
static void build_geometry_table(fem_mesh& m) {
    const HostLevel& L0 = m.lev[0];
    const int n0 = L0.n, N1 = n0 + 1;
    m.geo_ok = n0 <= kGeoMaxN;
    m.geo.clear();
    m.geo_count = 0;
    if (!m.geo_ok) return;
    const int64_t cnt = (int64_t)n0 * n0 * n0 * 36;
    m.geo_count = cnt;
    m.geo.assign((size_t)6 * cnt, 0.0);   // entries of one coarsest cube: 216 consecutive doubles
    auto edges = [](int t, double E[3][3]) {   // columns: V1 - V0, V2 - V0, V3 - V0 of path t
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) E[r][c] = 0.0;
        const int s0 = perm_axis(t, 0), s1 = perm_axis(t, 1);
        E[s0][0] = 1.0;
        E[s0][1] = 1.0;
        E[s1][1] = 1.0;
        for (int r = 0; r < 3; ++r) E[r][2] = 1.0;
    };
    for (int64_t q0 = 0; q0 < (int64_t)n0 * n0 * n0; ++q0) {
        const int ci = (int)(q0 % n0), cj = (int)((q0 / n0) % n0), ck = (int)(q0 / ((int64_t)n0 * n0));
        for (int t0 = 0; t0 < 6; ++t0) {
            const int s0 = perm_axis(t0, 0), s1 = perm_axis(t0, 1);
            int V[4][3] = {{ci, cj, ck}, {ci, cj, ck}, {ci, cj, ck}, {ci + 1, cj + 1, ck + 1}};
            V[1][s0] += 1;
            V[2][s0] += 1;
            V[2][s1] += 1;
            double X[4][3];
            for (int w = 0; w < 4; ++w) {
                const int64_t vid = V[w][0] + (int64_t)N1 * (V[w][1] + (int64_t)N1 * V[w][2]);
                for (int a = 0; a < 3; ++a) X[w][a] = L0.vxyz[3 * vid + a];
            }
            double J0[3][3], E0[3][3], Einv[3][3], Lm[3][3];
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) J0[r][c] = X[c + 1][r] - X[0][r];
            edges(t0, E0);
            // E0 is unimodular: its inverse is its adjugate times det (+-1), exact in doubles
            const double ed = E0[0][0] * (E0[1][1] * E0[2][2] - E0[1][2] * E0[2][1]) -
                              E0[0][1] * (E0[1][0] * E0[2][2] - E0[1][2] * E0[2][0]) +
                              E0[0][2] * (E0[1][0] * E0[2][1] - E0[1][1] * E0[2][0]);
            Einv[0][0] = (E0[1][1] * E0[2][2] - E0[1][2] * E0[2][1]) / ed;
            Einv[0][1] = (E0[0][2] * E0[2][1] - E0[0][1] * E0[2][2]) / ed;
            Einv[0][2] = (E0[0][1] * E0[1][2] - E0[0][2] * E0[1][1]) / ed;
            Einv[1][0] = (E0[1][2] * E0[2][0] - E0[1][0] * E0[2][2]) / ed;
            Einv[1][1] = (E0[0][0] * E0[2][2] - E0[0][2] * E0[2][0]) / ed;
            Einv[1][2] = (E0[0][2] * E0[1][0] - E0[0][0] * E0[1][2]) / ed;
            Einv[2][0] = (E0[1][0] * E0[2][1] - E0[1][1] * E0[2][0]) / ed;
            Einv[2][1] = (E0[0][1] * E0[2][0] - E0[0][0] * E0[2][1]) / ed;
            Einv[2][2] = (E0[0][0] * E0[1][1] - E0[0][1] * E0[1][0]) / ed;
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) {
                    double s = 0.0;
                    for (int k = 0; k < 3; ++k) s += J0[r][k] * Einv[k][c];
                    Lm[r][c] = s;
                }
            for (int t = 0; t < 6; ++t) {
                double E[3][3], M[3][3], g6[6];
                edges(t, E);
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c) {
                        double s = 0.0;
                        for (int k = 0; k < 3; ++k) s += Lm[r][k] * E[k][c];
                        M[r][c] = s;
                    }
                geometric_factor(M, g6);
                const int64_t idx = (q0 * 6 + t0) * 6 + t;
                for (int e = 0; e < 6; ++e) m.geo[(size_t)idx * 6 + e] = g6[e];
            }
        }
    }
    // Check: on every level, each cell's factors from its own vertex coordinates equal the table's
    // (up to the rounding of the midpoint coordinates), with the coarsest cell found as the
    // kernels find it, by ordering the centroid's coordinates inside the coarsest cube.
    for (int l = 0; l < m.nlev; ++l) {
        const HostLevel& L = m.lev[l];
        const int mask = (1 << l) - 1;
        const double scale = std::ldexp(1.0, -l);
        for (int64_t c = 0; c < L.C; ++c) {
            int V[4][3];
            cell_vertices(L, c, V);
            const int t = (int)((c % L.NC) / ((int64_t)L.B * L.B * L.B));
            int u[3];
            for (int a = 0; a < 3; ++a) u[a] = 4 * (V[0][a] & mask) + (V[1][a] - V[0][a]) + (V[2][a] - V[0][a]) + 1;
            int t0 = -1;
            for (int tt = 0; tt < 6; ++tt)
                if (u[perm_axis(tt, 0)] > u[perm_axis(tt, 1)] && u[perm_axis(tt, 1)] > u[perm_axis(tt, 2)]) t0 = tt;
            const int64_t q0 = (V[0][0] >> l) + (int64_t)n0 * ((V[0][1] >> l) + (int64_t)n0 * (V[0][2] >> l));
            const double* g = &m.geo[(size_t)((q0 * 6 + t0) * 6 + t) * 6];
            double gmax = 0.0, dmax = 0.0;
            for (int e = 0; e < 6; ++e) {
                const double ref = L.G64[(size_t)e * L.C + c];
                gmax = std::max(gmax, std::fabs(ref));
                dmax = std::max(dmax, std::fabs(ref - scale * g[e]));
            }
            if (t0 < 0 || !(dmax <= 1e-9 * gmax))
                throw std::runtime_error("geometry table does not match the cells of level " + std::to_string(l));
        }
    }
}

int action_geometry(const fem_mesh& m, int level) {
    const HostLevel& L = m.lev[level];
    // the cube kernel (P1/P2) and the lattice kernel (P3) on 4-cube bricks
    if (L.B != 4 || (L.p <= 2 && !L.cube)) return FEM_GEOM_CELL;
    // a 4-cube brick inside one coarsest cube: 2^level >= 4
    if (m.geo_ok && level >= 2) return FEM_GEOM_TABLE;
    return L.p <= 2 ? FEM_GEOM_VERTEX : FEM_GEOM_CELL;
}

// Structural check: every map entry equals the dof the brick reduction table expects.
static void validate_level(const HostLevel& L, const RedTable& t) {
    const int PB = L.p * L.B, QS = PB + 1;
    for (int64_t c = 0; c < L.C; ++c) {
        const int64_t brick = c / L.NC;
        const int cl = (int)(c % L.NC);
        const int bx = (int)(brick % L.nb), by = (int)((brick / L.nb) % L.nb), bz = (int)(brick / ((int64_t)L.nb * L.nb));
        for (int i = 0; i < L.nloc; ++i) {
            const int q = t.q_of[(size_t)cl * L.nloc + i];
            const int a = q % QS, b = (q / QS) % QS, cc = q / (QS * QS);
            const int64_t g = (bx * PB + a) + (int64_t)L.L * ((by * PB + b) + (int64_t)L.L * (bz * PB + cc));
            const uint32_t m = (uint32_t)L.map[(size_t)i * L.C + c] & ~kBoundaryBit;
            if ((int64_t)m != g) throw std::runtime_error("cell-to-dof map disagrees with the brick table");
        }
    }
}

static void build_tab(Tabulation& T, int p, int kvar) {
    const Rule& r = rule_for_degree(kvar ? 2 * p - 1 : 2 * p - 2);
    const int nl = nloc_of(p);
    T.p = p;
    T.kvar = kvar;
    T.nq = (int)r.w.size();
    if (T.nq != nq_of(p, kvar != 0)) throw std::runtime_error("quadrature size mismatch");
    T.stride = 1 + 4 + 3 * nl;
    T.t64.assign((size_t)T.nq * T.stride, 0.0);
    std::vector<double> dphi(nl * 3);
    for (int q = 0; q < T.nq; ++q) {
        double* o = &T.t64[(size_t)q * T.stride];
        o[0] = r.w[q];
        for (int v = 0; v < 4; ++v) o[1 + v] = r.lam[4 * q + v];
        eval_basis_grad(p, &r.x[3 * q], nullptr, dphi.data());
        for (int d = 0; d < 3; ++d)
            for (int i = 0; i < nl; ++i) o[5 + d * nl + i] = dphi[i * 3 + d];
    }
    T.t32.assign(T.t64.begin(), T.t64.end());
}

fem_status build_mesh(const fem_mesh_desc& d, fem_mesh& m) {
    m.desc = d;
    m.desc.jitter = nullptr;
    m.p = d.degree;
    m.nlev = d.n_refine + 1;
    const int p = d.degree;
    std::vector<std::array<int, 4>> mi;
    node_multi_indices(p, mi);
    m.lev.resize(m.nlev);
    for (int l = 0; l < m.nlev; ++l) {
        HostLevel& L = m.lev[l];
        L.n = d.n << l;
        L.p = p;
        L.nloc = nloc_of(p);
        const int n = L.n, N1 = n + 1;
        L.vxyz.assign((size_t)N1 * N1 * N1 * 3, 0.0);
        if (l == 0) {
            for (int k = 0; k < N1; ++k)
                for (int j = 0; j < N1; ++j)
                    for (int i = 0; i < N1; ++i) {
                        const size_t v = (size_t)i + N1 * ((size_t)j + N1 * k);
                        double x[3] = {(double)i / n, (double)j / n, (double)k / n};
                        const bool interior = i > 0 && j > 0 && k > 0 && i < n && j < n && k < n;
                        if ((d.flags & FEM_MESH_JITTER) && d.jitter && interior)
                            for (int a = 0; a < 3; ++a) x[a] += d.jitter[3 * v + a] / n;
                        for (int a = 0; a < 3; ++a) L.vxyz[3 * v + a] = x[a];
                    }
        } else {
            const HostLevel& Cc = m.lev[l - 1];
            const int nc1 = Cc.n + 1;
            for (int k = 0; k < N1; ++k)
                for (int j = 0; j < N1; ++j)
                    for (int i = 0; i < N1; ++i) {
                        const size_t v = (size_t)i + N1 * ((size_t)j + N1 * k);
                        const size_t lo = (size_t)(i / 2) + nc1 * ((size_t)(j / 2) + nc1 * (k / 2));
                        const size_t hi = (size_t)((i + 1) / 2) + nc1 * ((size_t)((j + 1) / 2) + nc1 * ((k + 1) / 2));
                        for (int a = 0; a < 3; ++a) L.vxyz[3 * v + a] = 0.5 * (Cc.vxyz[3 * lo + a] + Cc.vxyz[3 * hi + a]);
                    }
        }
        build_level(L, mi);
        L.red = find_red(m, p, L.B);
        L.red1 = find_red(m, 1, L.B);
        validate_level(L, m.red[L.red]);
        // the cube kernel addresses x, y and the coordinates with 32-bit byte offsets
        const bool fits = L.N * 8 < (1LL << 32) && 3 * L.NV * 8 < (1LL << 32);
        if (fits && L.B == 4 && p <= 2) build_cube_data(L);
        // interface slots: 8 side codes x the interface points of the degree-p and degree-1 lattices
        auto iface = [&](int po) {
            const int64_t Lo = (int64_t)po * L.n + 1, nb = L.nb, np = Lo - nb - 1;
            return (nb + 1) * Lo * Lo + (nb + 1) * np * Lo + (nb + 1) * np * np;
        };
        L.slot_elems = 8 * std::max(iface(p), iface(1));
    }
    for (int kv = 0; kv < 2; ++kv) build_tab(m.tab[kv], p, kv);
    build_geometry_table(m);
    build_transfer_tables(m);
    mass_matrix(p, m.mref64);
    m.mref32.assign(m.mref64.begin(), m.mref64.end());

    // device layout
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    for (auto& T : m.tab) {
        T.d64 = take(T.t64.size() * 8);
        T.d32 = take(T.t32.size() * 4);
    }
    m.d_mref64 = take(m.mref64.size() * 8);
    m.d_mref32 = take(m.mref32.size() * 4);
    m.d_geo = take(m.geo.size() * 8);
    m.d_pt_off = take(m.pt_off.size() * 4);
    m.d_pt_w64 = take(m.pt_w64.size() * 8);
    m.d_pt_w32 = take(m.pt_w32.size() * 4);
    m.d_rs_start = take(m.rs_start.size() * 4);
    m.d_rs_off = take(m.rs_off.size() * 4);
    m.d_rs_w64 = take(m.rs_w64.size() * 8);
    m.d_rs_w32 = take(m.rs_w32.size() * 4);
    for (auto& L : m.lev) {
        L.d_map = take(L.map.size() * 4);
        L.d_G64 = take(L.G64.size() * 8);
        L.d_G32 = take(L.G32.size() * 4);
        L.d_slots = take((size_t)L.slot_elems * 8);
        L.d_vsoa = take(L.vsoa.size() * 8);
        L.d_rs_lin = take(L.rs_lin.size() * 4);
    }
    m.bytes = off;
    return FEM_OK;
}

}  // namespace fem
