// Checks the per-face affine interface numbering used by the cube kernel's write-out against the
// point-wise numbering iface_index, and that every (slot plane, point) pair of a level is written
// by exactly the bricks that contain the point: for each brick, each of its closure points on a
// brick plane, the slot (code, t) lies inside the slot array, and no two (brick, point) pairs
// share a slot.  Built and run by tests/test_iface.py with the host C++ compiler.
#include <cstdio>
#include <vector>

#include "../paper_2104_08012_amd/csrc/iface.hpp"

template <int PB>
static int check(uint32_t nb) {
    const uint32_t L = PB * nb + 1, np = L - nb - 1;
    const uint32_t c0 = (nb + 1) * L * L, c01 = c0 + (nb + 1) * np * L, tot = c01 + (nb + 1) * np * np;
    std::vector<unsigned char> used((size_t)8 * tot, 0);
    int bad = 0;
    for (uint32_t bz = 0; bz < nb; ++bz)
        for (uint32_t by = 0; by < nb; ++by)
            for (uint32_t bx = 0; bx < nb; ++bx)
                for (uint32_t lc = 0; lc <= (uint32_t)PB; ++lc)
                    for (uint32_t lb = 0; lb <= (uint32_t)PB; ++lb)
                        for (uint32_t la = 0; la <= (uint32_t)PB; ++la) {
                            const bool fx = la == 0 || la == (uint32_t)PB, fy = lb == 0 || lb == (uint32_t)PB,
                                       fz = lc == 0 || lc == (uint32_t)PB;
                            if (!fx && !fy && !fz) continue;
                            const uint32_t I = bx * PB + la, J = by * PB + lb, K = bz * PB + lc;
                            const uint32_t t = fem::iface_index<PB>(I, J, K, L, nb, c0, c01);
                            uint32_t ta;
                            if (fx) ta = fem::iface_x0<PB>(bx, by, bz, la / PB, L) + lb + L * lc;
                            else if (fy) ta = fem::iface_y0<PB>(bx, by, bz, lb / PB, L, nb, c0) + la + np * lc;
                            else ta = fem::iface_z0<PB>(bx, by, bz, lc / PB, L, nb, c01) + la + np * lb;
                            const uint32_t code = (la == 0 ? 1u : 0u) | (lb == 0 ? 2u : 0u) | (lc == 0 ? 4u : 0u);
                            if (ta != t || t >= tot) { ++bad; continue; }
                            if (used[(size_t)code * tot + t]++) ++bad;
                        }
    return bad;
}

int main() {
    int bad = 0;
    for (uint32_t nb = 1; nb <= 5; ++nb)
        bad += check<1>(nb) + check<2>(nb) + check<4>(nb) + check<8>(nb) + check<12>(nb) + check<3>(nb);
    std::printf("%d\n", bad);
    return bad == 0 ? 0 : 1;
}
