// Compile-time incidence of lattice points in the six-tetrahedra cube split.
//
// A point of the P_p lattice (spacing h/p) is classified by its "type" (a mod p, b mod p,
// c mod p).  All points of one type meet the same cells at the same local nodes, up to a shift
// of the cube: a point of type (ta, tb, tc) in cube (X0, Y0, Z0) = floor(position / p) lies in
// the cubes X0 + dx with dx in {-1, 0} when ta == 0 and dx = 0 otherwise (likewise dy, dz), and in
// such a cube, at relative lattice position r = (ta - p dx, tb - p dy, tc - p dz), it is a node of
// the tetrahedron with axis order s exactly when r_s0 >= r_s1 >= r_s2, with barycentric
// multi-index m = (p - r_s0, r_s0 - r_s1, r_s1 - r_s2, r_s2).
//
// The table below lists, per type, every (dx, dy, dz, t, local node i) in a fixed order (dz, dy,
// dx outer to inner, then t).  It is built by constexpr evaluation, so the brick reduction
// compiles to straight-line code with no table loads.
#pragma once
#include "common.hpp"

namespace fem {

template <int P>
struct Incidence {
    static constexpr int NTYPE = P * P * P;
    static constexpr int MAXE = 24;
    int cnt[NTYPE];
    int dx[NTYPE][MAXE], dy[NTYPE][MAXE], dz[NTYPE][MAXE], t[NTYPE][MAXE], i[NTYPE][MAXE];

    static constexpr int node_index(int m0, int m1, int m2, int m3) {
        // local node order: vertices; edges (0,1),(0,2),(0,3),(1,2),(1,3),(2,3), each from its first
        // vertex towards its second; faces (0,1,2),(0,1,3),(0,2,3),(1,2,3)
        const int m[4] = {m0, m1, m2, m3};
        const int ea[6] = {0, 0, 0, 1, 1, 2}, eb[6] = {1, 2, 3, 2, 3, 3};
        for (int v = 0; v < 4; ++v)
            if (m[v] == P) return v;
        int idx = 4;
        for (int e = 0; e < 6; ++e)
            for (int s = 1; s < P; ++s, ++idx) {
                bool ok = m[ea[e]] == P - s && m[eb[e]] == s;
                for (int v = 0; v < 4; ++v)
                    if (v != ea[e] && v != eb[e] && m[v] != 0) ok = false;
                if (ok) return idx;
            }
        const int fa[4] = {0, 0, 0, 1}, fb[4] = {1, 1, 2, 2}, fc[4] = {2, 3, 3, 3};
        for (int f = 0; f < 4; ++f, ++idx) {
            bool ok = true;
            for (int v = 0; v < 4; ++v) {
                const bool on = (v == fa[f] || v == fb[f] || v == fc[f]);
                if ((on && m[v] != 1) || (!on && m[v] != 0)) ok = false;
            }
            if (ok) return idx;
        }
        return -1;
    }

    constexpr Incidence() : cnt{}, dx{}, dy{}, dz{}, t{}, i{} {
        for (int tc = 0; tc < P; ++tc)
            for (int tb = 0; tb < P; ++tb)
                for (int ta = 0; ta < P; ++ta) {
                    const int ty = ta + P * (tb + P * tc);
                    int n = 0;
                    for (int ddz = (tc == 0 ? -1 : 0); ddz <= 0; ++ddz)
                        for (int ddy = (tb == 0 ? -1 : 0); ddy <= 0; ++ddy)
                            for (int ddx = (ta == 0 ? -1 : 0); ddx <= 0; ++ddx) {
                                const int r[3] = {ta - P * ddx, tb - P * ddy, tc - P * ddz};
                                for (int tt = 0; tt < 6; ++tt) {
                                    const int s0 = perm_axis(tt, 0), s1 = perm_axis(tt, 1), s2 = perm_axis(tt, 2);
                                    if (r[s0] >= r[s1] && r[s1] >= r[s2]) {
                                        dx[ty][n] = ddx;
                                        dy[ty][n] = ddy;
                                        dz[ty][n] = ddz;
                                        t[ty][n] = tt;
                                        i[ty][n] = node_index(P - r[s0], r[s0] - r[s1], r[s1] - r[s2], r[s2]);
                                        ++n;
                                    }
                                }
                            }
                    cnt[ty] = n;
                }
    }
};

}  // namespace fem
