// Checks the interface numbering of iface.hpp for bricks of span PBX along x and PB along y, z:
//  1. the per-face affine indices equal the point-wise numbering, stay inside the slot array,
//     and give every (brick, face point) pair its own slot (every brick plane point of every
//     brick closure);
//  2. the write-out regions of the merged-brick cube kernel (R bricks of span PB along x in one
//     workgroup, wave w of R): the interior and the x-complete faces between the workgroup's
//     bricks go to y, the workgroup's faces to slots, so that every non-interface lattice point is
//     written to y exactly once, no interface point is, and every (workgroup brick, interface
//     point) pair gets exactly one slot.
// Built and run by tests/test_iface.py with the host C++ compiler.
#include <cstdio>
#include <vector>

#include "../paper_2104_08012_amd/csrc/iface.hpp"

template <int PBX, int PB>
static int check_numbering(uint32_t nbx, uint32_t nb) {
    const uint32_t L = PB * nb + 1, npx = L - nbx - 1;
    if (PBX * nbx + 1 != L) return 1;
    const fem::IfaceCounts ic = fem::iface_counts(L, nbx, nb);
    std::vector<unsigned char> used((size_t)8 * ic.total, 0);
    int bad = 0;
    for (uint32_t bz = 0; bz < nb; ++bz)
        for (uint32_t by = 0; by < nb; ++by)
            for (uint32_t bx = 0; bx < nbx; ++bx)
                for (uint32_t lc = 0; lc <= (uint32_t)PB; ++lc)
                    for (uint32_t lb = 0; lb <= (uint32_t)PB; ++lb)
                        for (uint32_t la = 0; la <= (uint32_t)PBX; ++la) {
                            const bool fx = la == 0 || la == (uint32_t)PBX, fy = lb == 0 || lb == (uint32_t)PB,
                                       fz = lc == 0 || lc == (uint32_t)PB;
                            if (!fx && !fy && !fz) continue;
                            const uint32_t I = bx * PBX + la, J = by * PB + lb, K = bz * PB + lc;
                            const uint32_t t = fem::iface_index<PBX, PB>(I, J, K, L, nbx, nb, ic.c0, ic.c01);
                            uint32_t ta;
                            if (fx) ta = fem::iface_x0<PBX, PB>(bx, by, bz, la / PBX, L) + lb + L * lc;
                            else if (fy) ta = fem::iface_y0<PBX, PB>(bx, by, bz, lb / PB, L, nbx, ic.c0) + la + npx * lc;
                            else ta = fem::iface_z0<PBX, PB>(bx, by, bz, lc / PB, L, nbx, nb, ic.c01) + la + npx * lb;
                            const uint32_t code = (la == 0 ? 1u : 0u) | (lb == 0 ? 2u : 0u) | (lc == 0 ? 4u : 0u);
                            if (ta != t || t >= ic.total) { ++bad; continue; }
                            if (used[(size_t)code * ic.total + t]++) ++bad;
                        }
    return bad;
}

// The merged-brick write-out: workgroup (px, by, bz), wave w of R handles brick-local la in
// [0, PB] of brick px R + w (pencil-local LA = w PB + la).
template <int PB, int R>
static int check_regions(uint32_t nbx) {
    constexpr int PBX = R * PB;
    const uint32_t nb = nbx * R, L = PB * nb + 1, npx = L - nbx - 1;
    const fem::IfaceCounts ic = fem::iface_counts(L, nbx, nb);
    std::vector<unsigned char> ywr((size_t)L * L * L, 0), used((size_t)8 * ic.total, 0);
    int bad = 0;
    auto slot = [&](uint32_t code, uint32_t t, uint32_t I, uint32_t J, uint32_t K) {
        if (t >= ic.total || t != fem::iface_index<PBX, PB>(I, J, K, L, nbx, nb, ic.c0, ic.c01)) { ++bad; return; }
        if (used[(size_t)code * ic.total + t]++) ++bad;
    };
    for (uint32_t bz = 0; bz < nb; ++bz)
        for (uint32_t by = 0; by < nb; ++by)
            for (uint32_t px = 0; px < nbx; ++px)
                for (int w = 0; w < R; ++w) {
                    const int la_lo = w == 0 ? 1 : 0;
                    // A: interior and the x-complete face la = 0 (w >= 1) to y
                    for (int lc = 1; lc < PB; ++lc)
                        for (int lb = 1; lb < PB; ++lb)
                            for (int la = la_lo; la < PB; ++la) {
                                const uint32_t I = px * PBX + w * PB + la, J = by * PB + lb, K = bz * PB + lc;
                                ywr[I + (size_t)L * (J + (size_t)L * K)]++;
                            }
                    // B: the workgroup's x faces (full faces), w = 0 lower, w = R - 1 upper
                    for (int sd = 0; sd < 2; ++sd) {
                        if ((sd == 0 && w != 0) || (sd == 1 && w != R - 1)) continue;
                        for (int lc = 0; lc <= PB; ++lc)
                            for (int lb = 0; lb <= PB; ++lb) {
                                const uint32_t t = fem::iface_x0<PBX, PB>(px, by, bz, sd, L) + lb + L * lc;
                                const uint32_t code = (sd == 0 ? 1u : 0u) | (lb == 0 ? 2u : 0u) | (lc == 0 ? 4u : 0u);
                                slot(code, t, (px + sd) * PBX, by * PB + lb, bz * PB + lc);
                            }
                    }
                    // C: y faces, la in [la_lo, PB - 1], all lc
                    for (int sd = 0; sd < 2; ++sd)
                        for (int lc = 0; lc <= PB; ++lc)
                            for (int la = la_lo; la < PB; ++la) {
                                const uint32_t LA = w * PB + la;
                                const uint32_t t = fem::iface_y0<PBX, PB>(px, by, bz, sd, L, nbx, ic.c0) + LA + npx * lc;
                                const uint32_t code = (sd == 0 ? 2u : 0u) | (lc == 0 ? 4u : 0u);
                                slot(code, t, px * PBX + LA, (by + sd) * PB, bz * PB + lc);
                            }
                    // D: z faces, la in [la_lo, PB - 1], lb inside
                    for (int sd = 0; sd < 2; ++sd)
                        for (int lb = 1; lb < PB; ++lb)
                            for (int la = la_lo; la < PB; ++la) {
                                const uint32_t LA = w * PB + la;
                                const uint32_t t = fem::iface_z0<PBX, PB>(px, by, bz, sd, L, nbx, nb, ic.c01) + LA + npx * lb;
                                slot(sd == 0 ? 4u : 0u, t, px * PBX + LA, by * PB + lb, (bz + sd) * PB);
                            }
                }
    // every non-interface point written to y once, no interface point; every slot of every
    // (workgroup brick, closure interface point) pair written once
    for (uint32_t K = 0; K < L; ++K)
        for (uint32_t J = 0; J < L; ++J)
            for (uint32_t I = 0; I < L; ++I) {
                const bool iface = I % PBX == 0 || J % PB == 0 || K % PB == 0;
                const unsigned char c = ywr[I + (size_t)L * (J + (size_t)L * K)];
                if (iface ? c != 0 : c != 1) ++bad;
                if (!iface) continue;
                const uint32_t t = fem::iface_index<PBX, PB>(I, J, K, L, nbx, nb, ic.c0, ic.c01);
                for (uint32_t code = 0; code < 8; ++code) {
                    bool exists = true;
                    const uint32_t X[3] = {I, J, K}, span[3] = {(uint32_t)PBX, (uint32_t)PB, (uint32_t)PB},
                                   nbd[3] = {nbx, nb, nb};
                    for (int d = 0; d < 3; ++d) {
                        const uint32_t q = X[d] / span[d], r = X[d] % span[d];
                        const bool hi = (code >> d) & 1u;
                        exists = exists && (hi ? (r == 0 && q < nbd[d]) : (r != 0 || q >= 1));
                    }
                    if ((used[(size_t)code * ic.total + t] != 0) != exists) ++bad;
                }
            }
    return bad;
}

int main() {
    int bad = 0;
    for (uint32_t nb = 1; nb <= 5; ++nb)
        bad += check_numbering<1, 1>(nb, nb) + check_numbering<2, 2>(nb, nb) + check_numbering<4, 4>(nb, nb) +
               check_numbering<8, 8>(nb, nb) + check_numbering<12, 12>(nb, nb) + check_numbering<3, 3>(nb, nb);
    for (uint32_t nbx = 1; nbx <= 3; ++nbx)
        bad += check_numbering<16, 8>(nbx, 2 * nbx) + check_numbering<32, 8>(nbx, 4 * nbx) +
               check_numbering<16, 4>(nbx, 4 * nbx) + check_numbering<8, 4>(nbx, 2 * nbx);
    for (uint32_t nbx = 1; nbx <= 3; ++nbx)
        bad += check_regions<8, 1>(nbx) + check_regions<8, 2>(nbx) + check_regions<8, 4>(nbx) +
               check_regions<4, 4>(nbx) + check_regions<4, 2>(nbx);
    std::printf("%d\n", bad);
    return bad == 0 ? 0 : 1;
}
