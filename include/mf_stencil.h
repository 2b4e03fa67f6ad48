/* mf_stencil.h — C ABI of the MI355X matrix-free P1 stencil library.
 *
 * The operator is the P1 finite-element Laplacian on a mesh of macro
 * triangles (2D) or tetrahedra (3D), each uniformly refined `level` times
 * (paper: Intro, "Hybrid Tetrahedral Grids"; the number of refinements is the
 * level).  Inside one macro every interior row of the matrix is the same
 * stencil — 7 points in 2D (the Vertex-to-Vertex kernel of the Performance
 * Modeling section), 15 points in 3D (the paper's stated next step in its
 * Conclusion and Outlook) — so the matrix is never stored (PETSc comparison
 * section, theoretical analysis).  Rows of DoFs on macro boundaries are
 * completed by interface handling between macros, which the paper assigns to
 * dedicated interface primitives rather than to the face kernels (Performance
 * Modeling, experiment description).  Domain-boundary DoFs get identity rows
 * (Dirichlet).
 *
 * Conventions shared by every call
 *  - All functions are extern "C", never throw, and return an int status
 *    (MF_OK = 0; negative = error, message in mf_last_error()).
 *  - Pointers named *_dev are device pointers on the current HIP device;
 *    host pointers are named without suffix.  `stream` is a hipStream_t
 *    (NULL = the default stream).  The caller owns every vector and workspace
 *    it passes; the library owns the mesh metadata (host and device) until
 *    destroy_macro_mesh.
 *  - Vectors are in STORAGE layout: the closed index space of every macro,
 *    concatenated in cell order.  In 2D the point (x, y), x, y >= 0,
 *    x + y <= N, N = 2^level, sits at y(N+2) - y(y+1)/2 + x of its macro (rows
 *    of N+1-y points, x fastest — the layout of the paper's generated
 *    vertex-to-vertex kernel).  In 3D slice z is the 2D triangle of side
 *    M = N - z, stored after slices 0..z-1: offset Tet(N+1) - Tet(N+1-z),
 *    Tet(n) = n(n+1)(n+2)/6.  DoFs on shared macro boundaries are stored once
 *    per macro; every function keeps all copies equal.
 *  - dtype MF_F64 = double vectors, MF_F32 = float vectors.
 *  - apply_stencil, smooth and residual (without a norm) are asynchronous on
 *    `stream`.  The mesh is read-only after creation, so calls on different
 *    streams with different buffers may overlap.
 */
#ifndef MF_STENCIL_H
#define MF_STENCIL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mf_mesh mf_mesh;

enum {
  MF_OK = 0,
  MF_NOT_CONVERGED = 1, /* vcycle_solve hit max_iter; x holds the last iterate */
  MF_EINVAL = -1,       /* bad argument: dim, null pointer, level range, degenerate or non-conforming mesh, dtype */
  MF_ENOMEM = -2,       /* host or device allocation failed, or a request exceeds a size limit */
  MF_EDEVICE = -3,      /* a HIP call failed; mf_last_error() holds hipGetErrorString */
  MF_ENOTSUP = -4,      /* valid but unsupported (e.g. device call on a host-only mesh) */
  MF_ENUMERIC = -5      /* a norm came out non-finite */
};

enum { MF_F64 = 0, MF_F32 = 1 };

enum {
  MF_FLAG_DIRICHLET = 1, /* bit0: every domain-boundary DoF is Dirichlet (identity row); set by default */
  MF_FLAG_HOST_ONLY = 2  /* bit1: build the host metadata only (no device memory); device calls return MF_ENOTSUP */
};

/* Thread-local message of the last error on this thread ("" if none). */
const char* mf_last_error(void);

/* Build a macro mesh and all per-level metadata up to max_level (0..15 in 2D,
 * 0..11 in 3D).
 *   coords: host, n_vertices*dim doubles.  cells: host, n_cells*(dim+1)
 *   vertex ids; the vertex order of a cell defines its index space
 *   (F(xi) = P0 + [P1-P0 | P2-P0 (| P3-P0)] xi, xi = lattice point / N).
 *   flags: MF_FLAG_* (pass MF_FLAG_DIRICHLET for the usual case).
 * Errors: MF_EINVAL for dim not 2/3, null pointers, vertex ids out of range,
 * a degenerate cell (|det J| <= 1e-14 * scale^dim), a repeated cell or a facet
 * shared by more than two cells; MF_ENOMEM / MF_EDEVICE on allocation or
 * upload failure.  On success *out owns host and device memory. */
int create_macro_mesh(int dim, int64_t n_vertices, const double* coords, int64_t n_cells,
                      const int64_t* cells, int max_level, int flags, mf_mesh** out);

/* Free everything the mesh owns.  NULL is accepted. */
int destroy_macro_mesh(mf_mesh* mesh);

/* Mesh facts: dimension, number of macros, maximum level. */
int mesh_info(const mf_mesh* mesh, int* dim, int64_t* n_macros, int* max_level);

/* Storage DoFs (length of a vector) and unique DoFs (shared copies counted once). */
int mesh_num_dofs(const mf_mesh* mesh, int level, int64_t* storage, int64_t* unique);

/* Exact integer key of every storage DoF (host arrays of storage*(dim+1)):
 * the (global vertex id, barycentric weight) pairs with non-zero weight,
 * sorted by vertex id, padded with (-1, 0).  Weights sum to N.  Copies of a
 * shared DoF have equal keys. */
int mesh_dof_keys(const mf_mesh* mesh, int level, int64_t* vids, int32_t* weights);

/* Storage index of n points given as (macro, x, y[, z]) rows (host arrays,
 * n*(dim+1) int64 in, n int64 out).  MF_EINVAL if a point lies outside its macro. */
int mesh_dof_index(const mf_mesh* mesh, int level, int64_t n, const int64_t* macro_lattice, int64_t* index);

/* The interior stencil of one macro at one level (host, 7 or 15 doubles).
 * 2D order: S, SE, W, C, E, NW, N (offsets (0,-1),(1,-1),(-1,0),(0,0),(1,0),(-1,1),(0,1)),
 * the weight order of the paper's generated vertex-to-vertex kernel.
 * 3D order: (0,0,-1),(1,0,-1),(0,1,-1),(-1,1,-1), the seven in-slice offsets
 * in the 2D order, then (0,-1,1),(1,-1,1),(-1,0,1),(0,0,1). */
int mesh_stencil(const mf_mesh* mesh, int level, int64_t macro, double* weights);

/* Bytes of device workspace vcycle_solve needs at `level` for a solver mode
 * (mf_solve_opts.mode, 0..5). */
int mesh_workspace_bytes(const mf_mesh* mesh, int level, int mode, int64_t* bytes);

/* Fill a storage vector with x = 2u - 1, u uniform in [0,1) from SplitMix64
 * (Steele, Lea, Flood, OOPSLA 2014) chained over (seed, key pairs): a seeded
 * U[-1,1) input that is equal on all copies of a shared DoF.  Asynchronous.
 * Test-input helper; no part of the operator. */
int mesh_fill_random(const mf_mesh* mesh, int level, int dtype, uint64_t seed, void* x_dev, void* stream);

/* y = b at Dirichlet DoFs (b_dev == NULL: y = 0 there); every other entry of
 * y is left unchanged.  Sets boundary values of a right-hand side or an
 * initial guess (the paper's benchmark problems fix Dirichlet values on the
 * domain boundary, Performance Modeling, Experiment Description).
 * Asynchronous. */
int mesh_set_dirichlet(const mf_mesh* mesh, int level, int dtype, const void* b_dev, void* y_dev, void* stream);

/* y = A x (paper: the "apply", i.e. an operator applied to a function,
 * Performance Modeling section).  Interior rows of each macro use its
 * constant stencil; macro-boundary rows are summed over the copies' partial
 * rows and written to every copy; Dirichlet rows give y = x.  y is
 * overwritten and must not alias x.  Asynchronous. */
int apply_stencil(const mf_mesh* mesh, int level, int dtype, const void* x_dev, void* y_dev, void* stream);

/* y = A(k) x for -div(k grad u) (P1), with k the P1 interpolant of the
 * nodal coefficient k_dev (storage layout of `level`, same dtype as x;
 * copies equal).  Each micro-triangle's (2D) or micro-tet's (3D) element
 * matrix is the mean of k over its vertices times the constant-coefficient
 * one, formed on the fly (no stored matrix: the paper's remark that varying
 * stencil weights can be computed on the fly, comparison of matrix-free and
 * sparse storage).  Dirichlet rows give y = x.  y is overwritten and must not
 * alias x or k.  Asynchronous. */
int apply_varcoef(const mf_mesh* mesh, int level, int dtype, const void* k_dev, const void* x_dev, void* y_dev,
                  void* stream);

/* y = A x on blended (non-affine) 2D macros, FP64: macro c maps its lattice
 * by F_c(xi) = P0 + (P1 - P0) xi1 + (P2 - P0) xi2 + xi0 xi1 xi2 d_c (xi =
 * lattice point / 2^level, xi0 = 1 - xi1 - xi2, P0..P2 its vertices in cell
 * order), a cubic bubble that vanishes on macro edges, so shared points
 * agree.  A is the P1 stiffness matrix of the straight micro-triangles on
 * the mapped points, with every element matrix formed on the fly (no two
 * rows share a stencil; the paper's remark that varying stencils can be
 * computed on the fly, comparison of matrix-free and sparse storage).
 * bubble_dev: n_macros x 2 doubles on the device (d_c).  Dirichlet rows give
 * y = x.  y must not alias x.  MF_ENOTSUP for a 3D mesh.  Asynchronous. */
int apply_blended(const mf_mesh* mesh, int level, const double* bubble_dev, const double* x_dev, double* y_dev,
                  void* stream);

/* y = A x for the P2 (quadratic) Laplace operator of a 2D mesh refined
 * `level` times: DoFs at the vertices and edge midpoints of the
 * micro-triangles (the paper's P2 discretisation, with its vertex-to-vertex,
 * edge-to-vertex, vertex-to-edge and edge-to-edge kernels of the
 * Performance Modeling section fused into one pass).  These DoFs are the
 * lattice points of level + 1, so x and y use the storage layout of level + 1
 * (mesh_num_dofs / mesh_dof_keys at level + 1); needs level + 1 <= max_level.
 * Rows: the assembled P2 stiffness matrix; Dirichlet rows give y = x.  y is
 * overwritten and must not alias x.  MF_ENOTSUP for a 3D mesh.  Asynchronous. */
int apply_p2(const mf_mesh* mesh, int level, int dtype, const void* x_dev, void* y_dev, void* stream);

/* `sweeps` weighted-Jacobi sweeps x <- x + omega D^-1 (b - A x) (the
 * multigrid smoother the paper names as a code-generated operation,
 * Performance Modeling section).  D is the assembled diagonal.  Dirichlet DoFs
 * are left unchanged.  tmp_dev is a vector of the same size used for
 * ping-pong; the result is in x_dev.  Asynchronous. */
int smooth(const mf_mesh* mesh, int level, int dtype, double omega, int sweeps, const void* b_dev,
           void* x_dev, void* tmp_dev, void* stream);

/* r = b - A x (Dirichlet rows: r = b - x).  If norm2 is non-NULL, also
 * ||r||_2 over unique DoFs, accumulated in FP64 in a fixed order (bitwise
 * reproducible); this synchronises `stream` and returns MF_ENUMERIC if the
 * norm is not finite. */
int residual(const mf_mesh* mesh, int level, int dtype, const void* b_dev, const void* x_dev, void* r_dev,
             double* norm2, void* stream);

/* residual() with the norm, for callers that cannot allocate device memory
 * (tight serving loops, harnesses that forbid hipMalloc): r = b - A x and
 * *norm2 = ||r||_2 over unique DoFs, the same kernels and bitwise the same
 * results as residual(..., norm2, ...).  The norm partials live in a static
 * device array of the library (2 MiB per device, held until the process
 * ends) instead of the mesh's buffers, so the call allocates nothing and
 * takes no lock.  Every call on one device shares that array: calls that
 * overlap on one device (other threads or streams) race and must be
 * serialised by the caller.  norm2 is required (host pointer); the call
 * synchronises `stream`.  MF_ENOMEM if the level's partials exceed the
 * array (more than 131,071 partial pairs: beyond the 2D level-14 triangle
 * or the 6-tet cube at level 9); MF_ENUMERIC if the norm is not finite. */
int residual_noalloc(const mf_mesh* mesh, int level, int dtype, const void* b_dev, const void* x_dev, void* r_dev,
                     double* norm2, void* stream);

/* Multigrid restriction r_c = P^T r_f from `level` to `level`-1, where P is
 * the P1 interpolation between the nested refinement levels (the paper
 * names the levels a natural basis for multigrid, Intro, "Hybrid Tetrahedral
 * Grids").  Each macro sums the fine values it owns (weight 1 at the
 * coincident point, 1/2 at the midpoints of the coarse micro-edges through
 * it), then copies of shared coarse DoFs are summed; Dirichlet coarse DoFs
 * get 0.  rf_dev: vector at `level`; bc_dev: vector at `level`-1
 * (overwritten).  level >= 1.  Asynchronous. */
int restrict_residual(const mf_mesh* mesh, int level, int dtype, const void* rf_dev, void* bc_dev, void* stream);

/* x_f += P e_c from `level`-1 to `level` (the interpolation above);
 * Dirichlet fine DoFs are left unchanged.  ec_dev: vector at `level`-1;
 * xf_dev: vector at `level`.  level >= 1.  Asynchronous. */
int prolong_add(const mf_mesh* mesh, int level, int dtype, const void* ec_dev, void* xf_dev, void* stream);

typedef struct {
  int mode;         /* 0: FP64 V-cycles in iterative refinement; 1: FP32 V-cycles in FP64 iterative
                       refinement; 2: conjugate gradients preconditioned by one FP64 V-cycle per
                       iteration; 3: the same with an FP32 V-cycle (FP64 recurrences); 4: MINRES
                       preconditioned by one FP64 V-cycle per iteration; 5: the same with an FP32
                       V-cycle (FP64 recurrences) */
  int pre, post;    /* smoothing sweeps (default 2, 2); modes 2 to 5 need pre == post (a symmetric
                       preconditioner), else MF_EINVAL */
  int coarse_level; /* solved directly (default min(2, level)) */
  int max_iter;     /* outer iterations (default 50) */
  double omega;     /* Jacobi weight (default 2/3) */
  double rtol;      /* stop when ||b - A x||_2 / ||b||_2 <= rtol over unique DoFs */
} mf_solve_opts;

typedef struct {
  int iters;
  double rel_res;
  double seconds;
} mf_solve_info;

/* Solve A x = b with V(pre,post)-cycles of geometric multigrid (levels are
 * the refinement hierarchy, Intro) as the correction of iterative refinement
 * (modes 0, 1), as the preconditioner of conjugate gradients (modes 2, 3;
 * every CG scalar stays on the device) or as the preconditioner of MINRES
 * (modes 4, 5: the Krylov method of the paper's plume application, section
 * Plume in Rectangular Domain; its scalars are formed on the host).  x_dev
 * holds the initial guess (its Dirichlet entries are set to b's);
 * workspace_dev must hold mesh_workspace_bytes(level, opts->mode) bytes.
 * The stopping test uses the true FP64 residual b - A x over unique DoFs:
 * recomputed each iteration in modes 0, 1; in modes 2 to 5 the Krylov
 * recurrence's residual (CG: its 2-norm; MINRES: sqrt(r . M r), M the
 * V-cycle, against its first value) decides when to recompute it,
 * and MF_OK is returned only if the recomputed one meets rtol (otherwise the
 * recurrence goes on).  info->rel_res is that true relative residual (modes 2
 * to 5 after a miss that ends at max_iter: the last recomputed one; MINRES
 * recomputes it at max_iter).  Returns MF_OK, MF_NOT_CONVERGED (x = last
 * iterate) or an error (MF_ENUMERIC if MINRES meets a preconditioner that is
 * not positive definite).  Synchronous; one device-to-host copy of two
 * doubles per iteration (MINRES: two), plus one per recomputed residual in
 * modes 2 to 5. */
int vcycle_solve(const mf_mesh* mesh, int level, const double* b_dev, double* x_dev, void* workspace_dev,
                 const mf_solve_opts* opts, mf_solve_info* info, void* stream);

/* Streaming device copy dst = src of n_bytes (a multiple of 16; both
 * pointers 16-byte aligned; no overlap): one 16-byte load and one
 * non-temporal 16-byte store per lane.  The measured copy bandwidth is the
 * reference the apply's HBM throughput is reported against, beside the
 * HBM3E peak (the paper measures its machine's load/store bandwidth the same
 * way before modelling its kernels, Intro, hardware description).  No part
 * of the operator.  Asynchronous. */
int device_copy(void* dst_dev, const void* src_dev, int64_t n_bytes, void* stream);

/* ---- Continuous batching of solves (serving) ----------------------------
 * A batch advances many independent solves of the kind vcycle_solve runs
 * (any meshes, dimensions and levels on the current device) together: each
 * batch_step performs one outer iteration for every member, and every kernel
 * of that iteration is launched once for all members that need it, its
 * workgroups dealt out among them.  The V-cycles of members of different
 * depth are aligned at their coarse level.  A member's arithmetic and its
 * order are those of vcycle_solve on its own, so its result is bitwise equal
 * to vcycle_solve with the same options.  This is the multigrid use of the
 * refinement levels (Intro, "Hybrid Tetrahedral Grids") applied to many
 * small problems at once, where single solves would be bound by launch
 * latency rather than by memory bandwidth. */
typedef struct mf_batch mf_batch;

/* opts: as for vcycle_solve (mode 0..3 only: MINRES is not batched; pre,
 * post, max_iter, omega; rtol is per member; coarse_level < 0 or above a
 * member's level selects min(2, level)).  NULL = mode 1, V(2,2), 50
 * iterations, omega 2/3; another mode is MF_EINVAL.  capacity: maximum members
 * (1..4096).  Allocates a small device table and pinned staging. */
int batch_create(const mf_solve_opts* opts, int capacity, mf_batch** out);
int batch_destroy(mf_batch* batch);
int batch_size(const mf_batch* batch, int* n);

/* Adds a solve of A x = b at `level` of `mesh`; x_dev holds the initial guess,
 * workspace_dev at least mesh_workspace_bytes(level, opts.mode) bytes.  The
 * caller keeps mesh, b, x and workspace alive and untouched until the member
 * is reported done.  tag identifies the member (unique within the batch).
 * MF_ENOMEM when the batch is full. */
int batch_add(mf_batch* batch, const mf_mesh* mesh, int level, const double* b_dev, double* x_dev,
              void* workspace_dev, double rtol, int64_t tag);

/* One outer iteration for every member (synchronises `stream` once).
 * Members that finished — converged (MF_OK), reached max_iter
 * (MF_NOT_CONVERGED) or met a non-finite norm (MF_ENUMERIC) — leave the
 * batch and are reported in done_tags / done_status / done_info (each with
 * room for batch_size() entries; done_info may be NULL); *n_done = their
 * number.  done_info.seconds = time since batch_add.  In modes 2, 3 a member
 * whose CG recurrence meets rtol spends its next step on recomputing the
 * true FP64 residual (no iteration), and finishes only if that meets rtol,
 * as vcycle_solve does. */
int batch_step(mf_batch* batch, void* stream, int64_t* done_tags, int* done_status, mf_solve_info* done_info,
               int* n_done);

#ifdef __cplusplus
}
#endif
#endif
