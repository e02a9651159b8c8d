// Numbering of the interface points of a brick decomposition (host and device).
//
// A level's output lattice has L points per direction (L = po n + 1) and nb bricks of PB = po B
// lattice spacings per direction.  Interface points are the lattice points on a brick plane
// (a coordinate that is a multiple of PB).  They are numbered family by family: points on x planes
// first, then points on y planes but no x plane, then points on z planes only:
//   x planes: t = (I / PB) L^2 + K L + J
//   y planes: t = c0 + (J / PB) np L + K np + iu           (iu: rank of I among non-plane values)
//   z planes: t = c01 + (K / PB) np^2 + ju np + iu
// with np = L - nb - 1 non-plane coordinates per direction, c0 = (nb + 1) L^2 and
// c01 = c0 + (nb + 1) np L.  A brick's contribution to point t is stored at slot
// code * total + t, code = sum_d [the brick is the upper one along d] << d.
#pragma once
#include <cstdint>

#include "common.hpp"

namespace fem {

template <int PB>
FEM_HD inline uint32_t iface_index(uint32_t I, uint32_t J, uint32_t K, uint32_t L, uint32_t nb, uint32_t c0,
                                   uint32_t c01) {
    const uint32_t np = L - nb - 1;
    if (I % PB == 0) return (I / PB) * L * L + K * L + J;
    const uint32_t iu = (I / PB) * (PB - 1) + I % PB - 1;
    if (J % PB == 0) return c0 + (J / PB) * np * L + K * np + iu;
    const uint32_t ju = (J / PB) * (PB - 1) + J % PB - 1;
    return c01 + (K / PB) * np * np + ju * np + iu;
}

// Within one face of brick (bx, by, bz) the index is affine in the two in-face coordinates.
// s = 0 for the lower face along the axis, 1 for the upper one; la, lb, lc are brick-local.
//   x face (la = s PB, all lb, lc):               t = iface_x0 + lb + L lc
//   y face (lb = s PB, 1 <= la < PB, all lc):      t = iface_y0 + la + np lc
//   z face (lc = s PB, 1 <= la, lb < PB):          t = iface_z0 + la + np lb
template <int PB>
FEM_HD inline uint32_t iface_x0(uint32_t bx, uint32_t by, uint32_t bz, uint32_t s, uint32_t L) {
    return (bx + s) * L * L + bz * PB * L + by * PB;
}
template <int PB>
FEM_HD inline uint32_t iface_y0(uint32_t bx, uint32_t by, uint32_t bz, uint32_t s, uint32_t L, uint32_t nb,
                                uint32_t c0) {
    const uint32_t np = L - nb - 1;
    return c0 + (by + s) * np * L + bz * PB * np + bx * (PB - 1) - 1;
}
template <int PB>
FEM_HD inline uint32_t iface_z0(uint32_t bx, uint32_t by, uint32_t bz, uint32_t s, uint32_t L, uint32_t nb,
                                uint32_t c01) {
    const uint32_t np = L - nb - 1;
    return c01 + (bz + s) * np * np + (by * (PB - 1) - 1) * np + bx * (PB - 1) - 1;
}

}  // namespace fem
