// Vertex stars of the cube split on the P_p lattice (p = 2, 3), as compile-time tables.
//
// Section 2, Listing 2 smooths with the patch preconditioner over star patches around mesh
// vertices (construct_type star, construct_dim 0): the star of vertex v holds the dofs carried by
// the entities whose closure contains v.  In a cell where v is local vertex i these are the nodes
// with barycentric multi-index m_i > 0.  With vertex v at lattice point p V (V its integer vertex
// coordinates), a node of a cell with integer vertices W_w sits at lattice point sum_w m_w W_w,
// so the star is described by the lattice offsets of its nodes from p V:
//   p = 2: 1 vertex + 14 edge midpoints (the 14 edge directions of the split): 15 dofs;
//   p = 3: 1 vertex + 28 edge nodes (two per edge) + 36 face nodes (one per triangle around v):
//          65 dofs.
// Slot numbering.  p = 2 keeps the numbering of the P2 kernels: slot 0 the vertex, slot c (1..7)
// the offset d(c) = (c & 1, (c >> 1) & 1, c >> 2), slot 7 + c the offset -d(c).  p = 3 numbers
// the offsets in lexicographic order (z, then y, then x) of the 5^3 box [-2, 2]^3.
// Every cell around v is the tetrahedron t of the cube whose corner o (bits x, y, z) is v, when
// that corner is one of t's four path vertices; the tables list, per (o, t), the local vertex
// index of v, the cell's star nodes and their slots.
// Gathering the star results per dof: a dof at lattice point X lies in the cube floor(X / p) at
// residue r = X mod p; the tetrahedron whose path follows the decreasing order of r's components
// holds it with multi-index m = (p - r_s0, r_s0 - r_s1, r_s1 - r_s2, r_s2); the stars holding the
// dof are those of the path vertices with m_w > 0, listed by increasing vertex index.
#pragma once
#include "common.hpp"
#include "tabulate.hpp"

namespace fem {

template <int P>
struct StarTab {
    static constexpr int NS = P == 2 ? 15 : 65;       // dofs of an interior star
    static constexpr int NP = NS * (NS + 1) / 2;      // packed lower triangle
    static constexpr int NCN = P == 2 ? 4 : 10;       // star nodes of one cell (m_i > 0)
    static constexpr int NL = nloc_of(P);
    int off[NS][3];          // lattice offset of each slot from p V
    int slot[5][5][5];       // offset + 2 -> slot, -1 outside the star
    int iv[8][6];            // local index of v in tetrahedron t of the cube with v at corner o, or -1
    int cn[8][6][NCN];       // that cell's star nodes (local node indices)
    int cs[8][6][NCN];       // their slots
    int rn[P][P][P];         // residue class -> number of stars holding the dof (1..3)
    int rv[P][P][P][3];      // corner bits of each star's vertex in the dof's cube, increasing index
    int rs[P][P][P][3];      // slot of the dof in that star

    constexpr StarTab() : off{}, slot{}, iv{}, cn{}, cs{}, rn{}, rv{}, rs{} {
        const NodeList<P> nodes{};
        for (int a = 0; a < 5; ++a)
            for (int b = 0; b < 5; ++b)
                for (int c = 0; c < 5; ++c) slot[a][b][c] = -1;
        // offsets of all cells' star nodes
        bool seen[5][5][5] = {};
        for (int o = 0; o < 8; ++o)
            for (int t = 0; t < 6; ++t) {
                int V[4][3] = {};
                path(t, V);
                iv[o][t] = -1;
                for (int w = 0; w < 4; ++w)
                    if (V[w][0] == (o & 1) && V[w][1] == ((o >> 1) & 1) && V[w][2] == (o >> 2)) iv[o][t] = w;
                if (iv[o][t] < 0) continue;
                int k = 0;
                for (int i = 0; i < NL; ++i) {
                    if (nodes.m[i][iv[o][t]] == 0) continue;
                    int X[3] = {0, 0, 0};
                    for (int w = 0; w < 4; ++w)
                        for (int d = 0; d < 3; ++d) X[d] += nodes.m[i][w] * V[w][d];
                    const int ox = X[0] - P * (o & 1), oy = X[1] - P * ((o >> 1) & 1), oz = X[2] - P * (o >> 2);
                    seen[ox + 2][oy + 2][oz + 2] = true;
                    cn[o][t][k++] = i;
                }
            }
        if (P == 2) {
            for (int c = 0; c < 8; ++c) {
                const int dx = c & 1, dy = (c >> 1) & 1, dz = c >> 2;
                set_slot(c, dx, dy, dz);
                if (c > 0) set_slot(7 + c, -dx, -dy, -dz);
            }
        } else {
            int s = 0;
            for (int oz = -2; oz <= 2; ++oz)
                for (int oy = -2; oy <= 2; ++oy)
                    for (int ox = -2; ox <= 2; ++ox)
                        if (seen[ox + 2][oy + 2][oz + 2] && s < NS) set_slot(s++, ox, oy, oz);
        }
        for (int o = 0; o < 8; ++o)
            for (int t = 0; t < 6; ++t) {
                if (iv[o][t] < 0) continue;
                int V[4][3] = {};
                path(t, V);
                for (int k = 0; k < NCN; ++k) {
                    int X[3] = {0, 0, 0};
                    for (int w = 0; w < 4; ++w)
                        for (int d = 0; d < 3; ++d) X[d] += nodes.m[cn[o][t][k]][w] * V[w][d];
                    cs[o][t][k] = slot[X[0] - P * (o & 1) + 2][X[1] - P * ((o >> 1) & 1) + 2][X[2] - P * (o >> 2) + 2];
                }
            }
        // residue classes
        for (int rx = 0; rx < P; ++rx)
            for (int ry = 0; ry < P; ++ry)
                for (int rz = 0; rz < P; ++rz) {
                    const int r[3] = {rx, ry, rz};
                    int t = 0;
                    for (int tt = 0; tt < 6; ++tt)
                        if (r[perm_axis(tt, 0)] >= r[perm_axis(tt, 1)] && r[perm_axis(tt, 1)] >= r[perm_axis(tt, 2)]) {
                            t = tt;
                            break;
                        }
                    const int s0 = perm_axis(t, 0), s1 = perm_axis(t, 1), s2 = perm_axis(t, 2);
                    const int m[4] = {P - r[s0], r[s0] - r[s1], r[s1] - r[s2], r[s2]};
                    int V[4][3] = {};
                    path(t, V);
                    // path vertices have increasing corner bits, so w order is increasing vertex index
                    int k = 0;
                    for (int w = 0; w < 4; ++w) {
                        if (m[w] == 0) continue;
                        const int bits = V[w][0] + 2 * V[w][1] + 4 * V[w][2];
                        rv[rx][ry][rz][k] = bits;
                        rs[rx][ry][rz][k] = slot[r[0] - P * V[w][0] + 2][r[1] - P * V[w][1] + 2][r[2] - P * V[w][2] + 2];
                        ++k;
                    }
                    rn[rx][ry][rz] = k;
                }
    }
    constexpr void set_slot(int s, int ox, int oy, int oz) {
        off[s][0] = ox;
        off[s][1] = oy;
        off[s][2] = oz;
        slot[ox + 2][oy + 2][oz + 2] = s;
    }
    static constexpr void path(int t, int (&V)[4][3]) {
        for (int w = 0; w < 4; ++w)
            for (int d = 0; d < 3; ++d) V[w][d] = 0;
        V[1][perm_axis(t, 0)] = 1;
        V[2][perm_axis(t, 0)] = 1;
        V[2][perm_axis(t, 1)] = 1;
        V[3][0] = V[3][1] = V[3][2] = 1;
    }
    // checks used by static_assert: every offset present was given a slot, every slot is
    // distinct, every cell's star nodes have slots, residue classes hold 1 to 3 stars
    constexpr int count_slots() const {
        int n = 0;
        for (int a = 0; a < 5; ++a)
            for (int b = 0; b < 5; ++b)
                for (int c = 0; c < 5; ++c) n += slot[a][b][c] >= 0;
        return n;
    }
    constexpr int cells_around() const {
        int n = 0;
        for (int o = 0; o < 8; ++o)
            for (int t = 0; t < 6; ++t) n += iv[o][t] >= 0;
        return n;
    }
    constexpr bool consistent() const {
        for (int o = 0; o < 8; ++o)
            for (int t = 0; t < 6; ++t)
                if (iv[o][t] >= 0)
                    for (int k = 0; k < NCN; ++k)
                        if (cs[o][t][k] < 0 || cs[o][t][k] >= NS) return false;
        for (int rx = 0; rx < P; ++rx)
            for (int ry = 0; ry < P; ++ry)
                for (int rz = 0; rz < P; ++rz) {
                    const int n = rn[rx][ry][rz];
                    if (n < 1 || n > 3) return false;
                    for (int k = 0; k < n; ++k)
                        if (rs[rx][ry][rz][k] < 0) return false;
                    for (int k = 1; k < n; ++k)
                        if (rv[rx][ry][rz][k] <= rv[rx][ry][rz][k - 1]) return false;
                }
        return true;
    }
};

static_assert(StarTab<2>{}.count_slots() == 15 && StarTab<2>{}.cells_around() == 24 && StarTab<2>{}.consistent(),
              "P2 star: 15 dofs from the 24 cells around a vertex");
static_assert(StarTab<3>{}.count_slots() == 65 && StarTab<3>{}.cells_around() == 24 && StarTab<3>{}.consistent(),
              "P3 star: 65 dofs (vertex, 2 per edge on 14 edges, 36 faces) from the 24 cells around a vertex");

}  // namespace fem
