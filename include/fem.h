/*
 * fem.h - C ABI of the MI355X (gfx950) matrix-free Poisson / multigrid-CG library.
 *
 * The library applies the operator of the weak form
 *     a(u, v) = int_Omega k grad(u) . grad(v) dx                (paper Section 2, eq. 4)
 * for continuous Lagrange P1-P3 elements (Section 2, Listing 1: FunctionSpace(mesh, "CG", degree))
 * on a tetrahedral unit cube refined uniformly (Listing 1: UnitCubeMesh, MeshHierarchy), with
 * homogeneous Dirichlet conditions on all six faces (Listing 1: DirichletBC), and solves
 * A u = b by conjugate gradients preconditioned with a geometric multigrid V-cycle whose levels
 * are smoothed by two Chebyshev iterations and whose coarsest level is solved directly
 * (Section 4, Listing 2).  k is either 1 (the paper's problem) or a continuous piecewise-linear
 * field given by its vertex values.  It also computes dJ/dk for J = 1/2 ||u - u_obs||^2_{L2} by
 * the adjoint method (the sensitivities motivated in Section 1).
 *
 * Conventions
 *  - Every entry point returns fem_status: 0 = FEM_OK, > 0 warning, < 0 error.  Arguments are
 *    validated on the host before anything is enqueued; a call that returns an error has
 *    enqueued nothing (a solve may leave x holding its last iterate).  fem_last_error() gives a
 *    per-thread message for the most recent failure.
 *  - Device pointers are plain pointers into caller-owned device memory; "stream" is a
 *    hipStream_t passed as void* (NULL = the default stream).  The library never allocates
 *    memory visible to the caller: mesh data and solver workspaces live in caller buffers sized
 *    by the *_bytes queries (256-byte aligned) that must outlive the handles using them.
 *  - Vectors are in the library's dof order: the P_p dofs of level l sit on the lattice of
 *    spacing h_l / p, and dof (I, J, K) has index I + L (J + L K), L = p n_l + 1.  Vertex
 *    fields (k, dJ/dk) use the vertex lattice: index i + (n_l+1) (j + (n_l+1) k).
 *  - Level 0 is the coarsest mesh; level n_refine the finest.
 *  - Apply, mass, diagonal, transfer and gradient calls are stream-ordered and asynchronous.
 *    Solver calls are host-synchronous (they take convergence decisions on the host).
 *  - Calls that use the same mesh level (or the same solver workspace) on different streams
 *    concurrently race: each level owns one interface scratch area inside the mesh buffer.
 */
#ifndef FEM_H
#define FEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fem_status;
enum {
    FEM_OK = 0,
    FEM_WARN_NOT_CONVERGED = 1,
    FEM_ERR_INVALID_ARG = -1,
    FEM_ERR_UNSUPPORTED = -2,
    FEM_ERR_WORKSPACE = -3,
    FEM_ERR_HIP = -4,
    FEM_ERR_BREAKDOWN = -5,
    FEM_ERR_STATE = -6
};

typedef enum { FEM_F64 = 0, FEM_F32 = 1 } fem_dtype;

/* flags for the operator applications */
enum {
    FEM_BC_IDENTITY = 0,  /* y = P_I A P_I x + P_B x: identity rows/zero columns on boundary dofs */
    FEM_BC_NONE = 1,      /* y = A x, the raw operator (A . 1 = 0 for the stiffness operator)  */
    FEM_BC_ZERO_ROWS = 2  /* y = P_I A x: boundary rows zeroed, columns kept                     */
};

/* mesh description */
enum { FEM_MESH_JITTER = 1u };
typedef struct {
    int32_t n;              /* cubes per direction of the coarsest mesh (>= 1)            */
    int32_t n_refine;       /* uniform refinements; levels = n_refine + 1 (<= 7)           */
    int32_t degree;         /* Lagrange degree p in {1, 2, 3}                              */
    uint32_t flags;         /* FEM_MESH_JITTER: move coarsest interior vertices             */
    const double* jitter;   /* host, ((n+1)^3, 3) offsets in units of h = 1/n, x fastest;
                               read only when FEM_MESH_JITTER is set; boundary rows ignored */
} fem_mesh_desc;

/* Where the stiffness action of a level takes its geometry from (fem_level_info.geometry). */
enum {
    FEM_GEOM_CELL = 0,    /* per-cell factors G stored for every cell (P3, bricks below 4 cubes) */
    FEM_GEOM_VERTEX = 1,  /* the vertex coordinates, G formed in the kernel (P1/P2, 4-cube bricks) */
    FEM_GEOM_TABLE = 2    /* the coarsest level's table of G per (coarsest cell, tetrahedron type),
                             scaled by 2^-level: P1/P2 levels whose 4-cube bricks each lie in one
                             coarsest cube, coarsest mesh of at most 24^3 cubes.  Every level is a
                             uniform refinement of the coarsest, affine on each coarsest cell. */
};

typedef struct {
    int64_t n_cells, n_dofs, n_interior, n_vertices;
    int32_t n, degree, brick;   /* cubes per direction, degree, cubes per brick edge */
    int32_t geometry;           /* FEM_GEOM_* of the stiffness action on this level */
} fem_level_info;

typedef struct fem_mesh fem_mesh;

/* Build a mesh hierarchy on the host: topology, numbering, per-cell geometric factors
 * G = |det J| J^-1 J^-T, cell-to-dof maps, brick reduction and transfer tables.
 * Section 2, Listing 1 (UnitCubeMesh, MeshHierarchy, FunctionSpace).  Host only.
 * Errors: FEM_ERR_INVALID_ARG (NULL, n < 1, degree outside 1..3, a level with 2^29 cells or
 *         dofs or more: the kernels use 32-bit byte offsets per array),
 *         FEM_ERR_INVALID_ARG when jitter inverts a cell. */
fem_status fem_mesh_create(const fem_mesh_desc* desc, fem_mesh** out);

/* Bytes of the device buffer the mesh needs (256-byte multiple). Host only. */
fem_status fem_mesh_device_bytes(const fem_mesh* mesh, size_t* bytes);

/* Copy the mesh to a caller-owned device buffer of at least fem_mesh_device_bytes bytes on the
 * current HIP device.  Blocks until the copy is complete.  The buffer must outlive the mesh.
 * Errors: FEM_ERR_INVALID_ARG (NULL, misaligned), FEM_ERR_WORKSPACE (too small), FEM_ERR_HIP. */
fem_status fem_mesh_upload(fem_mesh* mesh, void* device_buffer, size_t bytes, void* stream);

fem_status fem_mesh_levels(const fem_mesh* mesh, int32_t* n_levels);
fem_status fem_mesh_info(const fem_mesh* mesh, int32_t level, fem_level_info* info);

/* Lattice coordinates of every dof of a level: host array (3 * n_dofs) int32, (I, J, K) per dof. */
fem_status fem_mesh_dof_lattice(const fem_mesh* mesh, int32_t level, int32_t* ijk);

/* Vertex positions of a level: host array (3 * n_vertices) double. */
fem_status fem_mesh_vertex_coords(const fem_mesh* mesh, int32_t level, double* xyz);

void fem_mesh_destroy(fem_mesh* mesh);

/* y = A(k) x, the matrix-free stiffness action on one level (Section 2, eq. 4; the element
 * integrals use a quadrature rule exact for the polynomial integrand: degree 2p-2 for k = 1,
 * 2p-1 for P1 k).  k_vertex: NULL for k = 1, else n_vertices values of dtype.  x, y: n_dofs
 * values of dtype, device, x != y.  flags: FEM_BC_IDENTITY | FEM_BC_NONE | FEM_BC_ZERO_ROWS.
 * Stream-ordered.  Deterministic: the scatter-add runs in a fixed order.
 * Errors: FEM_ERR_INVALID_ARG, FEM_ERR_STATE (mesh not uploaded), FEM_ERR_HIP. */
fem_status fem_apply_laplacian(const fem_mesh* mesh, int32_t level, fem_dtype dtype,
                               const void* k_vertex, const void* x, void* y,
                               uint32_t flags, void* stream);

/* y = alpha * A(k) x + beta * z (z may equal y; z ignored when beta == 0). Same layout rules. */
fem_status fem_apply_laplacian_axpby(const fem_mesh* mesh, int32_t level, fem_dtype dtype,
                                     const void* k_vertex, const void* x, double alpha,
                                     const void* z, double beta, void* y,
                                     uint32_t flags, void* stream);

/* For callers that cannot allocate device memory or have it allocated for them (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): y = A(k) x exactly as
 * fem_apply_laplacian computes it (the same kernels; the same result bit for bit), except that the
 * kernels keep the interface partial sums of the brick decomposition in a library-owned
 * file-scope device array of 64 MiB per GPU instead of the level's slot area in the mesh buffer.
 * Allocates nothing: the array's device address is looked up once per GPU on the first call made
 * with that GPU current.  Arguments as fem_apply_laplacian; the current device must be the one
 * the mesh was uploaded to.  The array needs 8 * (interface points) * sizeof(dtype) bytes for the
 * level (P2 up to 64^3 cubes in FP64, P3 up to 48^3); larger levels return FEM_ERR_WORKSPACE
 * before anything is enqueued.  Every call on a GPU shares that GPU's array and leaves its partial
 * sums there (no call reads a value it has not written first, so nothing needs clearing); calls
 * that overlap in time on one GPU (other streams, concurrent graph replays) race on the array.
 * Stream-ordered.  Errors: FEM_ERR_INVALID_ARG (as fem_apply_laplacian, or another device
 * current), FEM_ERR_STATE, FEM_ERR_WORKSPACE, FEM_ERR_HIP. */
fem_status fem_apply_laplacian_noalloc(const fem_mesh* mesh, int32_t level, fem_dtype dtype,
                                       const void* k_vertex, const void* x, void* y,
                                       uint32_t flags, void* stream);

/* y = M x, the consistent mass matrix int phi_i phi_j (used for J and the adjoint right-hand
 * side).  flags as above (FEM_BC_NONE gives the raw matrix). */
fem_status fem_apply_mass(const fem_mesh* mesh, int32_t level, fem_dtype dtype,
                          const void* x, void* y, uint32_t flags, void* stream);

/* d = diag(A_bc(k)) (boundary entries 1), the Jacobi scaling of the Chebyshev smoother
 * (Section 4, Listing 2). */
fem_status fem_assemble_diagonal(const fem_mesh* mesh, int32_t level, fem_dtype dtype,
                                 const void* k_vertex, void* d, void* stream);

/* Multigrid transfers between level fine_level-1 and fine_level (Section 4: nested spaces
 * from uniform refinement).  Prolongation: x_fine += P x_coarse (P interpolates the coarse
 * function at the fine nodes).  Restriction: r_coarse = P^T r_fine with boundary rows zeroed. */
fem_status fem_prolong(const fem_mesh* mesh, int32_t fine_level, fem_dtype dtype,
                       const void* x_coarse, void* x_fine, void* stream);
fem_status fem_restrict(const fem_mesh* mesh, int32_t fine_level, fem_dtype dtype,
                        const void* r_fine, void* r_coarse, void* stream);

/* Assembled operator (the representation of the paper's solvers, §4: a sparse matrix and SpMV),
 * for comparison with the matrix-free action.  fem_csr_create builds on the host the CSR pattern of
 * A_bc on one level (rows and columns in the library's dof order; int32 row pointers and columns)
 * and, for every stored entry, the list of element-matrix entries summed into it, in ascending cell
 * order.  fem_csr_upload copies pattern and lists into a caller-owned device buffer of
 * device_bytes (256-byte aligned; it also holds the FP64 element-matrix scratch of
 * C * nloc^2 doubles).  fem_csr_assemble forms the element matrices of A(k) (same quadrature as
 * the matrix-free action; k_vertex: NULL for k = 1 or FP64 device vertex values) and sums them in
 * that fixed order into values (nnz entries of dtype, caller-owned device memory): Dirichlet rows
 * become identity rows and Dirichlet columns zero.  fem_csr_spmv: y = A x (n_rows entries of dtype,
 * x != y), bitwise reproducible.  Levels whose C * nloc^2 or nnz reach 2^31 are
 * FEM_ERR_UNSUPPORTED. */
typedef struct fem_csr fem_csr;
fem_status fem_csr_create(const fem_mesh* mesh, int32_t level, fem_csr** out);
fem_status fem_csr_info(const fem_csr* a, int64_t* n_rows, int64_t* nnz, size_t* device_bytes);
fem_status fem_csr_pattern(const fem_csr* a, int32_t* row_ptr_host, int32_t* col_host);
fem_status fem_csr_upload(fem_csr* a, void* device, size_t bytes, void* stream);
fem_status fem_csr_assemble(fem_csr* a, fem_dtype dtype, const double* k_vertex, void* values, void* stream);
fem_status fem_csr_spmv(const fem_csr* a, fem_dtype dtype, const void* values, const void* x, void* y,
                        void* stream);
void fem_csr_destroy(fem_csr* a);

/* Solver */
enum { FEM_PREC_FP64 = 0, FEM_PREC_MIXED = 1 };
/* Coarse solve (Section 4, Listing 2: a direct solve on the coarsest level, mg_coarse_pc_type lu).
 * AUTO: the dense FP64 inverse up to 40,000 interior coarse dofs, else nested FP64 MG-PCG to
 * coarse_rtol over the levels below.  DENSE / NESTED force one of the two.  DENSE_F32 (mixed
 * precision only; FEM_ERR_INVALID_ARG otherwise): the dense inverse computed in FP64 but stored in
 * FP32 (products accumulated in FP64): a relaxation of the exact FP64 coarse solve that halves
 * its bytes, available only when asked for. */
enum { FEM_COARSE_AUTO = 0, FEM_COARSE_DENSE = 1, FEM_COARSE_NESTED = 2, FEM_COARSE_DENSE_F32 = 3 };
enum { FEM_PC_MG = 0, FEM_PC_JACOBI = 1 };
enum { FEM_SMOOTHER_JACOBI = 0, FEM_SMOOTHER_PATCH = 1 };

typedef struct {
    double rtol;                 /* stop when ||b - A x|| / ||b|| <= rtol                       */
    int32_t max_it;              /* outer CG iterations                                         */
    int32_t precision;           /* FEM_PREC_FP64 or FEM_PREC_MIXED                             */
    int32_t n_levels_used;       /* levels in the outer V-cycle (0 = all); the lowest of them is
                                    solved directly, or by nested FP64 MG-PCG over the levels below */
    int32_t cheb_degree;         /* Chebyshev steps per smoothing (Listing 2: 2)                */
    double cheb_lo, cheb_hi;     /* interval [lo, hi] * lambda_max of D^-1 A                     */
    int32_t eig_iters;           /* Lanczos steps for lambda_max                               */
    int32_t coarse_method;       /* FEM_COARSE_*                                                */
    const double* lambda_max_override; /* host, NULL or one value per mesh level (0 = estimate) */
    double coarse_rtol;          /* nested coarse solve tolerance                               */
    int32_t replace_every;       /* true-residual replacement period (0 = never)               */
    int32_t flexible;            /* 1: Polak-Ribiere beta                                       */
    double* history;             /* host, may be NULL: relative residual per iteration          */
    int32_t history_cap;
    int32_t preconditioner;      /* FEM_PC_MG (V-cycle) or FEM_PC_JACOBI (diag(A)^-1 on the finest level) */
    int32_t level_timing;        /* 1: record HIP events around every level of every V-cycle and
                                    report fem_solve_stats.level_ms (costs a few microseconds per
                                    level transition); 0 (default): level_ms stay zero            */
    int32_t smoother;            /* preconditioner of the Chebyshev smoother on the smoothed levels:
                                    FEM_SMOOTHER_JACOBI (default, diag(A)^-1) or FEM_SMOOTHER_PATCH
                                    (Listing 2: additive vertex-star patches, degrees 2 and 3, as
                                    fem_apply_patch; lambda_max of B_patch A from CG-Lanczos).  A
                                    nested coarse solver smooths with Jacobi.                     */
} fem_solve_opts;

typedef struct {
    int32_t iterations;
    int32_t coarse_iterations;   /* nested coarse solver iterations, summed                  */
    double rel_residual_true;    /* ||b - A x|| / ||b|| in FP64 at exit                        */
    double setup_ms, solve_ms, coarse_ms; /* coarse_ms: with level_timing = 1                   */
    double level_ms[8];          /* time spent per mesh level in the V-cycles (level_timing = 1) */
    double lambda_max[8];
} fem_solve_stats;

void fem_solve_opts_default(fem_solve_opts* opts);

typedef struct fem_solver fem_solver;

/* Workspace bytes for a solver on this mesh with these options (256-byte multiple). */
fem_status fem_solve_workspace_bytes(const fem_mesh* mesh, const fem_solve_opts* opts, size_t* bytes);

/* A solver handle binds mesh, options and a caller-owned device workspace. */
fem_status fem_solver_create(const fem_mesh* mesh, const fem_solve_opts* opts,
                             void* workspace, size_t ws_bytes, fem_solver** out);
/* Per-coefficient setup: injected k on every level, Jacobi diagonals, lambda_max by Lanczos,
 * coarse operator and its dense inverse (or nested solver).  k_vertex: NULL (k = 1) or FP64
 * device array on the finest level's vertices.  Host-synchronous. */
fem_status fem_solver_setup(fem_solver* s, const double* k_vertex, void* stream);
/* Solve A_bc(k) x = b, the discrete Poisson problem of Section 2 (eq. 4 with Listing 1's
 * Dirichlet conditions), by CG preconditioned with the multigrid cycle of Section 4, Listing 2
 * (Chebyshev smoothing, direct coarse solve) until ||b - A x|| / ||b|| <= rtol.  b, x: FP64
 * device, finest level, n_dofs each, caller-owned; x in: initial guess, out: solution.
 * Host-synchronous.  Returns FEM_WARN_NOT_CONVERGED when max_it is reached (x holds the last
 * iterate), FEM_ERR_BREAKDOWN on p^T A p <= 0 or non-finite scalars, FEM_ERR_STATE before
 * fem_solver_setup. */
fem_status fem_solver_solve(fem_solver* s, const double* b, double* x, fem_solve_stats* stats, void* stream);
/* z = B r: one application of the multigrid preconditioner (FP64 in/out, finest level). */
fem_status fem_solver_vcycle(fem_solver* s, const double* r, double* z, void* stream);
/* One full-multigrid cycle as the solver (Listing 2: pc_mg_type full with a preonly outer
 * solver): b (FP64 device, finest level, boundary rows zero) is restricted to every level used,
 * the coarsest is solved exactly, and on each finer level the prolonged solution is corrected by
 * one V-cycle on that level's residual; x (FP64 device, overwritten) receives the finest-level
 * result.  In mixed precision the V-cycles run in FP32 (restriction, prolongation, residuals and
 * the coarse solve stay FP64).  stats: iterations = 1, rel_residual_true = ||b - A x|| / ||b||,
 * solve_ms.  Host-synchronous; needs the multigrid preconditioner (FEM_ERR_UNSUPPORTED for
 * Jacobi). */
fem_status fem_solver_fmg(fem_solver* s, const double* b, double* x, fem_solve_stats* stats, void* stream);
/* Switch the per-level timing of later solves on (1) or off (0), as fem_solve_opts.level_timing
 * does at creation.  FEM_ERR_INVALID_ARG for a NULL solver. */
fem_status fem_solver_set_level_timing(fem_solver* s, int32_t on);
void fem_solver_destroy(fem_solver* s);

/* One-shot solve of A_bc(k) x = b (Section 2 eq. 4 with Listing 1's boundary conditions; the
 * multigrid-preconditioned CG of Section 4, Listing 2): create a solver on the caller's
 * workspace (ws_bytes >= fem_solve_workspace_bytes), set it up for k_vertex (NULL => k = 1, else
 * FP64 device values on the finest level's vertices), solve and destroy it.  b, x as in
 * fem_solver_solve; stats (host, may be NULL) receives iterations, residual and times.  Errors
 * and warnings as fem_solver_create, fem_solver_setup and fem_solver_solve. */
fem_status fem_mg_cg_solve(const fem_mesh* mesh, const double* k_vertex, const double* b, double* x,
                           const fem_solve_opts* opts, void* workspace, size_t ws_bytes,
                           fem_solve_stats* stats, void* stream);

/* Adjoint gradient of a functional of the solution with respect to the vertex values of k (the
 * sensitivities of Section 1, for the operator of Section 2 eq. 4 with a P1 coefficient):
 *     grad_v = - sum_K int_K psi_v grad(u) . grad(lambda) dx   over the cells K containing v,
 * psi_v the P1 hat function, i.e. -d(lambda^T A(k) u)/dk_v; with lambda the adjoint solution
 * (A_bc lambda = dJ/du) this is dJ/dk_v.  u, lambda: FP64 device, n_dofs of `level`; grad: FP64
 * device, n_vertices, overwritten; all caller-owned.  k_vertex is accepted for symmetry with the
 * solve and not read (A is linear in k).  Stream-ordered.  Errors: FEM_ERR_INVALID_ARG (NULL
 * pointers, level out of range), FEM_ERR_STATE (mesh not uploaded), FEM_ERR_HIP. */
fem_status fem_adjoint_grad_k(const fem_mesh* mesh, int32_t level, const double* k_vertex,
                              const double* u, const double* lambda, double* grad, void* stream);

/* Additive vertex-star patch preconditioner (Section 2, Listing 2: the smoother's preconditioner
 * is the patch preconditioner with star patches around vertices, construct_dim 0):
 *     z = sum_v R_v^T A_v^{-1} R_v r on interior dofs,  z_B = r_B,
 * R_v restricting to the interior dofs whose carrying entity contains vertex v, A_v = R_v A R_v^T
 * with A the stiffness matrix of k.  Degrees 2 and 3: an interior star holds 15 dofs for P2 (the
 * vertex and the 14 edge midpoints around it) and 65 for P3 (the vertex, two dofs on each of 14
 * edges, one on each of 36 faces).  Degree 1 (every star one dof: point Jacobi) and levels whose
 * packed index (entries per vertex x n_vertices rounded up to 64) reaches 2^32 return
 * FEM_ERR_UNSUPPORTED.
 * fem_patch_bytes: size of the caller-owned patch buffer of `level` for dtype (the packed
 * lower triangles of the star inverses, 120 (P2) or 2145 (P3) entries per vertex, plus 15 or 65
 * partial results per vertex, over the vertex count rounded up to a multiple of 64), 256-byte
 * aligned parts.
 * fem_patch_setup: fills the buffer for k_vertex (FP64 device, n_vertices; NULL => k = 1); the
 * inverses are computed in FP64 and stored in dtype.  FEM_ERR_WORKSPACE for a NULL or short
 * buffer.  Stream-ordered.
 * fem_apply_patch: z = B_patch r (r, z device, n_dofs of `level`, dtype; z overwritten, z != r).
 * Writes the partial-result part of the buffer, so two applications that share one buffer must
 * not run concurrently.  Stream-ordered. */
fem_status fem_patch_bytes(const fem_mesh* mesh, int32_t level, fem_dtype dtype, size_t* bytes);
fem_status fem_patch_setup(const fem_mesh* mesh, int32_t level, fem_dtype dtype, const double* k_vertex,
                           void* patch, size_t bytes, void* stream);
fem_status fem_apply_patch(const fem_mesh* mesh, int32_t level, fem_dtype dtype, void* patch, size_t bytes,
                           const void* r, void* z, void* stream);

const char* fem_status_string(fem_status s);
const char* fem_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FEM_H */
