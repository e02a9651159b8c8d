// temporary
#include "internal.hpp"
extern "C" {
void fem_solve_opts_default(fem_solve_opts* o) { (void)o; }
fem_status fem_solve_workspace_bytes(const fem_mesh*, const fem_solve_opts*, size_t*) { return FEM_ERR_UNSUPPORTED; }
fem_status fem_solver_create(const fem_mesh*, const fem_solve_opts*, void*, size_t, fem_solver**) { return FEM_ERR_UNSUPPORTED; }
fem_status fem_solver_setup(fem_solver*, const double*, void*) { return FEM_ERR_UNSUPPORTED; }
fem_status fem_solver_solve(fem_solver*, const double*, double*, fem_solve_stats*, void*) { return FEM_ERR_UNSUPPORTED; }
fem_status fem_solver_vcycle(fem_solver*, const double*, double*, void*) { return FEM_ERR_UNSUPPORTED; }
void fem_solver_destroy(fem_solver*) {}
fem_status fem_mg_cg_solve(const fem_mesh*, const double*, const double*, double*, const fem_solve_opts*, void*, size_t, fem_solve_stats*, void*) { return FEM_ERR_UNSUPPORTED; }
}
