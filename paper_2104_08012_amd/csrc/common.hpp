// Constants shared by the host code and the gfx950 kernels of the library.
#pragma once
#include <cstdint>

#if defined(__HIPCC__)
#define FEM_HD __host__ __device__
#else
#define FEM_HD
#endif

namespace fem {

// Local dofs of Lagrange P_p on a tetrahedron: (p+1)(p+2)(p+3)/6.
FEM_HD constexpr int nloc_of(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }

// Quadrature points per cell.  Stiffness with k = 1 has integrand degree 2p-2, with a P1
// coefficient (and the adjoint gradient, which carries one P1 factor) degree 2p-1.
//   degree <= 1: 1 point (centroid)   degree 2: 4 points   degree 3: 5 points
//   degree 4: 11 points               degree 5: 14 points
FEM_HD constexpr int nq_of(int p, bool kvar) {
    return p == 1 ? 1 : p == 2 ? (kvar ? 5 : 4) : (kvar ? 14 : 11);
}

// Six tetrahedra per cube, one per axis order s (lexicographic order of the permutations of
// {0,1,2}); the cell's vertices follow the monotone lattice path
//   v0 = c, v1 = v0 + e_s0, v2 = v1 + e_s1, v3 = c + (1,1,1).
FEM_HD constexpr int perm_axis(int t, int k) {
    // t = 0..5 : (0,1,2) (0,2,1) (1,0,2) (1,2,0) (2,0,1) (2,1,0)
    return (t == 0) ? k : (t == 1) ? (k == 0 ? 0 : k == 1 ? 2 : 1)
         : (t == 2) ? (k == 0 ? 1 : k == 1 ? 0 : 2) : (t == 3) ? (k == 0 ? 1 : k == 1 ? 2 : 0)
         : (t == 4) ? (k == 0 ? 2 : k == 1 ? 0 : 1) : (k == 0 ? 2 : k == 1 ? 1 : 0);
}

// Coarsest levels up to this many cubes per direction carry the hierarchy's geometry table.
constexpr int kGeoMaxN = 24;

// Centroid of path tetrahedron t of the unit cube, times 4: 3, 2, 1 along axes s0, s1, s2.
FEM_HD constexpr int centroid4(int t, int d) {
    return perm_axis(t, 0) == d ? 3 : perm_axis(t, 1) == d ? 2 : 1;
}
// The type of the path tetrahedron holding a point with pairwise distinct coordinates u, from
// the bits [u0 > u1] + 2 [u0 > u2] + 4 [u1 > u2]: three bits per code, packed.
FEM_HD constexpr int path_type_code() {
    int code = 0;
    for (int t = 0; t < 6; ++t) {
        const int u0 = centroid4(t, 0), u1 = centroid4(t, 1), u2 = centroid4(t, 2);
        code |= t << (3 * ((u0 > u1) + 2 * (u0 > u2) + 4 * (u1 > u2)));
    }
    return code;
}
constexpr int kPathTypeCode = path_type_code();

// The boundary flag of a dof lives in the sign bit of the cell-to-dof map entry.
constexpr uint32_t kBoundaryBit = 0x80000000u;

// Geometric factor storage order (symmetric 3x3): 00, 11, 22, 01, 02, 12.
enum { G00 = 0, G11 = 1, G22 = 2, G01 = 3, G02 = 4, G12 = 5 };

// Cell-wise operations that scatter-add into shared dofs.
enum Kind : int { K_APPLY = 0, K_DIAG = 1, K_MASS = 2, K_GRAD = 4 };

// Row treatment of boundary dofs in scatter kernels.
enum RowMode : int { ROW_NONE = 0, ROW_IDENTITY = 1, ROW_ZERO = 2, ROW_ONE = 3 };

}  // namespace fem
