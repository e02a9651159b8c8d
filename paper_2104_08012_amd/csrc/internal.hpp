// Internal host-side data structures of the library.
#pragma once
#include <array>
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fem.h"
#include "common.hpp"

namespace fem {

// ---------------- reference element (refelem.cpp) ----------------
struct Rule {
    std::vector<double> x;    // nq * 3 reference coordinates
    std::vector<double> lam;  // nq * 4 barycentric coordinates
    std::vector<double> w;    // nq weights (sum 1/6)
    int degree = 0;
};
void node_multi_indices(int p, std::vector<std::array<int, 4>>& out);
void eval_basis_grad(int p, const double xi[3], double* phi, double* dphi);
void mass_matrix(int p, std::vector<double>& M);
const Rule& rule_for_degree(int degree);
double rule_exactness_error(int degree);

// ---------------- error reporting (capi.cpp) ----------------
void set_error(const std::string& msg);

// ---------------- mesh (mesh.cpp) ----------------
inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Brick reduction table: for a brick of B^3 cubes (6 B^3 cells) and output nodes of degree po,
// the closure points q of the brick's po-lattice box (Q = (po B + 1)^3), for each the list of
// (local node i, local cell cl) contributions as LDS offsets i * NC + cl, in a fixed order,
// and the compact slot of q among the brick-boundary points (-1 for points inside the brick).
struct RedTable {
    int po = 0, B = 0, NC = 0, Q = 0, QB = 0;
    std::vector<int32_t> off, ent, slot;
    std::vector<int32_t> q_of;  // (cl * nloc(po) + i) -> q, used by the host validation
};

// Quadrature tabulation for the stiffness-type kernels of degree p:
// per point q: w_q, lambda_q[4], D_q[3][nloc] (reference gradients of the basis).
struct Tabulation {
    int p = 0, kvar = 0, nq = 0, stride = 0;
    std::vector<double> t64;
    std::vector<float> t32;
    size_t d64 = 0, d32 = 0;
};

struct HostLevel {
    int n = 0, p = 0, nloc = 0, B = 0, nb = 0, NC = 0, L = 0;
    int64_t C = 0, N = 0, NI = 0, NV = 0, nbricks = 0;
    std::vector<double> vxyz;      // NV * 3
    std::vector<int32_t> map;      // SoA nloc * C, sign bit = boundary dof
    std::vector<double> G64;       // SoA 6 * C
    std::vector<float> G32;
    // Cube-kernel data (P1/P2 on 4-cube bricks, whose dofs are addressed by their lattice point):
    // the vertex coordinates SoA (x[NV], y[NV], z[NV]) in FP64.
    bool cube = false;
    std::vector<double> vsoa;
    int red = -1, red1 = -1;       // reduction tables for degree p and for degree 1 output
    int64_t slot_elems = 0;        // interface partial slots (max over the tables used)
    std::vector<int32_t> rs_lin;   // restriction onto this level: stencil offsets as linear offsets
                                   // on the next finer level's lattice (entry order of rs_off)
    size_t d_map = 0, d_G64 = 0, d_G32 = 0, d_slots = 0, d_vsoa = 0, d_rs_lin = 0;
};

}  // namespace fem

struct fem_mesh {
    fem_mesh_desc desc{};
    int p = 0, nlev = 0;
    std::vector<fem::HostLevel> lev;
    std::vector<fem::RedTable> red;
    fem::Tabulation tab[2];          // [kvar]
    // geometric factors of the whole hierarchy from the coarsest level (every level is a uniform
    // refinement of it, so the mesh is affine on each coarsest tetrahedron): for coarsest cube q0,
    // coarsest tetrahedron type t0 and fine tetrahedron type t, G(L E_t) with L the coarsest
    // cell's lattice-to-physical map and E_t the lattice edges of type t; a tetrahedron of type t
    // on level l inside that coarsest cell has G = 2^-l G(L E_t).  Entry e (00, 11, 22, 01, 02,
    // 12) of index (q0 * 6 + t0) * 6 + t at 6 * index + e, so one coarsest cube's 216 values are
    // consecutive.  Built when the coarsest level has at most kGeoMaxN^3 cubes (geo_ok).
    bool geo_ok = false;
    int64_t geo_count = 0;
    std::vector<double> geo;
    size_t d_geo = 0;
    std::vector<double> mref64;      // nloc * nloc
    std::vector<float> mref32;
    size_t d_mref64 = 0, d_mref32 = 0;
    // lattice transfers (transfer.cpp): prolongation weights per local fine position (pt_ne
    // entries each: packed node offset, weight) and restriction stencils per residue class
    int pt_ne = 0;
    std::vector<int32_t> pt_off, rs_start, rs_off;
    std::vector<double> pt_w64, rs_w64;
    std::vector<float> pt_w32, rs_w32;
    size_t d_pt_off = 0, d_pt_w64 = 0, d_pt_w32 = 0, d_rs_start = 0, d_rs_off = 0, d_rs_w64 = 0, d_rs_w32 = 0;
    size_t bytes = 0;
    char* dev = nullptr;
    int device = -1;
};

namespace fem {
fem_status build_mesh(const fem_mesh_desc& d, fem_mesh& m);
void build_transfer_tables(fem_mesh& m);
// FEM_GEOM_* of the stiffness action on a level (the kernel choice of the launcher)
int action_geometry(const fem_mesh& m, int level);
}
