// Numbering of the interface points of a brick decomposition (host and device).
//
// A level's output lattice has L points per direction (L = po n + 1).  Bricks span PBX lattice
// spacings along x and PB along y and z (PBX = R PB when R bricks of the kernel's workgroup are
// merged along x; PBX = PB otherwise), with nbx and nb bricks per direction.  Interface points
// are the lattice points on a brick plane (I a multiple of PBX, or J or K a multiple of PB).
// They are numbered family by family: points on x planes first, then points on y planes but no
// x plane, then points on z planes only:
//   x planes: t = (I / PBX) L^2 + K L + J
//   y planes: t = c0 + (J / PB) L npx + K npx + iu          (iu: rank of I among non-x-plane values)
//   z planes: t = c01 + (K / PB) np npx + ju npx + iu       (ju: rank of J among non-y-plane values)
// with npx = L - nbx - 1, np = L - nb - 1, c0 = (nbx + 1) L^2, c01 = c0 + (nb + 1) L npx and
// total = c01 + (nb + 1) np npx.  A brick's contribution to point t is stored at slot
// code * total + t, code = sum_d [the brick is the upper one along d] << d.
#pragma once
#include <cstdint>

#include "common.hpp"

namespace fem {

struct IfaceCounts {
    uint32_t c0, c01, total;
};

FEM_HD inline IfaceCounts iface_counts(uint32_t L, uint32_t nbx, uint32_t nb) {
    const uint32_t npx = L - nbx - 1, np = L - nb - 1;
    IfaceCounts c;
    c.c0 = (nbx + 1) * L * L;
    c.c01 = c.c0 + (nb + 1) * L * npx;
    c.total = c.c01 + (nb + 1) * np * npx;
    return c;
}

template <int PBX, int PB>
FEM_HD inline uint32_t iface_index(uint32_t I, uint32_t J, uint32_t K, uint32_t L, uint32_t nbx, uint32_t nb,
                                   uint32_t c0, uint32_t c01) {
    const uint32_t npx = L - nbx - 1, np = L - nb - 1;
    if (I % PBX == 0) return (I / PBX) * L * L + K * L + J;
    const uint32_t iu = (I / PBX) * (PBX - 1) + I % PBX - 1;
    if (J % PB == 0) return c0 + (J / PB) * L * npx + K * npx + iu;
    const uint32_t ju = (J / PB) * (PB - 1) + J % PB - 1;
    return c01 + (K / PB) * np * npx + ju * npx + iu;
}

// Within one face of a brick the index is affine in the two in-face coordinates.  The brick has
// lattice origin (ox, oy, oz) = (bx PBX, by PB, bz PB) along x, y, z in units of its own spans
// (bx counts bricks of span PBX); s = 0 for the lower face along the axis, 1 for the upper one;
// la, lb, lc are brick-local (la in [0, PBX]).
//   x face (la = s PBX, all lb, lc):                   t = iface_x0 + lb + L lc
//   y face (lb = s PB, 1 <= la < PBX, all lc):          t = iface_y0 + la + npx lc
//   z face (lc = s PB, 1 <= la < PBX, 1 <= lb < PB):    t = iface_z0 + la + npx lb
template <int PBX, int PB>
FEM_HD inline uint32_t iface_x0(uint32_t bx, uint32_t by, uint32_t bz, uint32_t s, uint32_t L) {
    return (bx + s) * L * L + bz * PB * L + by * PB;
}
template <int PBX, int PB>
FEM_HD inline uint32_t iface_y0(uint32_t bx, uint32_t by, uint32_t bz, uint32_t s, uint32_t L, uint32_t nbx,
                                uint32_t c0) {
    const uint32_t npx = L - nbx - 1;
    return c0 + (by + s) * L * npx + bz * PB * npx + bx * (PBX - 1) - 1;
}
template <int PBX, int PB>
FEM_HD inline uint32_t iface_z0(uint32_t bx, uint32_t by, uint32_t bz, uint32_t s, uint32_t L, uint32_t nbx,
                                uint32_t nb, uint32_t c01) {
    const uint32_t npx = L - nbx - 1, np = L - nb - 1;
    return c01 + (bz + s) * np * npx + (by * (PB - 1) - 1) * npx + bx * (PBX - 1) - 1;
}

}  // namespace fem
