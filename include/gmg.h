/*
 * gmg.h -- C ABI of an MI355X (gfx950) implementation of adaptive geometric
 * multigrid with local smoothing for Q_k finite elements on 2:1-balanced
 * quad/hex forests (Clevenger, Heister, Kanschat, Kronbichler,
 * arXiv:1904.03317).
 *
 * What is solved (Sec. 2.1): find u in V_h, the conforming Q_k space on the
 * leaf mesh with hanging nodes eliminated (Sec. 2.3) and u = 0 on the domain
 * boundary, such that  sum_K a_K int_K grad u . grad v = int f_h v  for all v,
 * with a cell-wise constant coefficient a_K (Sec. 4.3) and f_h the nodal
 * interpolant of the given nodal values.  The method (Sec. 1, 2.2, 2.3, 4.1):
 * conjugate gradients in FP64, preconditioned by one V-cycle (Alg. 2) with
 * local smoothing on the level meshes, a Chebyshev-Jacobi smoother (Alg. 1
 * with Chebyshev acceleration), transfer operators that are the embedding and
 * its Euclidean adjoint, and an exact coarse solve.  The V-cycle runs in FP32
 * or FP64 (mixed precision as in Sec. 4.1).
 *
 * Conventions
 *  - Every call returns int: 0 = OK, GMG_NOT_CONVERGED (+1) = solve finished
 *    without reaching the tolerance (outputs are still written), negative =
 *    error.  gmg_last_error() returns a thread-local message for the last
 *    failing call on this thread.  No C++ exception crosses this ABI.
 *  - Pointers named d_* are device pointers (HIP device memory of the current
 *    device); all other pointers are host pointers.  The caller owns every
 *    buffer it passes in.  Arrays returned through gmg_problem_array() are
 *    owned by the library and stay valid until the problem is destroyed.
 *  - Device work is ordered on the caller's stream; calls that return host
 *    results (solve, vcycle timings, bind) synchronise that stream first.
 *  - Geometry: coarse cells are unit squares/cubes [o, o+1]^d at distinct
 *    integer origins o.  A cell of level l has side 2^-l; anchors are given in
 *    global integer units of 2^-20.  Maximum level 16.
 *  - Canonical cell order: by coarse cell, then z-order (Morton, child id
 *    x + 2y + 4z) of the anchor -- depth-first order of the forest.
 *  - A level DoF flag is 0 = S (smoothed on this level), 1 = I (interface:
 *    node of a level-l cell lying in the closure of a coarser leaf), 2 = D
 *    (on the domain boundary).  Sec. 2.3, Fig. 1.
 */
#ifndef GMG_H
#define GMG_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  GMG_OK = 0,
  GMG_NOT_CONVERGED = 1,
  GMG_E_INVAL = -1,
  GMG_E_NOMEM_HOST = -2,
  GMG_E_NOMEM_DEVICE = -3,
  GMG_E_BUDGET = -4,
  GMG_E_BREAKDOWN = -5,
  GMG_E_NAN = -6,
  GMG_E_HIP = -7,
  GMG_E_STATE = -8
};

typedef struct gmg_mesh_s* gmg_mesh;
typedef struct gmg_problem_s* gmg_problem;
typedef struct gmg_server_s* gmg_server;

/* Solver options.  Defaults from gmg_options_default(): degree 2, FP32
 * V-cycle, Chebyshev smoother of degree 4 on [0.08, 1.2] * lambda_max
 * (Sec. 4.1), 10 eigenvalue-estimate iterations (Sec. 4.1), rtol 1e-10 on
 * the unpreconditioned residual (Sec. 4.1, 4.3), max_iter 100, relax 1. */
typedef struct {
  int32_t degree;        /* k = 1..4 */
  int32_t mg_precision;  /* 32: FP32 V-cycle inside FP64 CG; 64: FP64 throughout */
  int32_t cheb_degree;   /* smoothing steps per smoother call, >= 1 */
  double cheb_lo;        /* lower end of the damped range, fraction of lambda_max */
  double cheb_hi;        /* upper end, fraction of lambda_max */
  int32_t eig_iters;     /* CG steps of the lambda_max estimate */
  double rtol;           /* stop when ||b - A u||_2 <= rtol ||b||_2 */
  int32_t max_iter;      /* CG iteration cap */
  int32_t use_graph;     /* 1: replay the V-cycle as a captured HIP graph */
  int32_t op_variant;    /* level operator form; 0 (the only value): sibling-family patches on
                            levels >= 1 in the entity layout (GMG_ARR_LEVEL_PERM) */
  int32_t smoother;      /* GMG_SMOOTHER_CHEBYSHEV (Sec. 4.1) or GMG_SMOOTHER_JACOBI: cheb_degree
                            steps of x += relax D^{-1} (g - A x) (Sec. 4.3 "MF": one step, relax 1) */
  double relax;          /* Jacobi relaxation factor, 0 < relax <= 2 */
} gmg_options;

enum { GMG_SMOOTHER_CHEBYSHEV = 0, GMG_SMOOTHER_JACOBI = 1 };

void gmg_options_default(gmg_options* opts);
const char* gmg_last_error(void);

/* ---------------------------------------------------------------- forest
 * Sec. 2.2 (mesh hierarchy by isotropic refinement), Sec. 2.3 (forest,
 * levels, leaf mesh), Sec. 3.5 (2:1 balance).  Host only. */

/* New forest of level-0 leaves.  origins: [n_coarse * dim] integer origins,
 * distinct.  dim in {2,3}; 1 <= n_coarse <= 128, within a box of 16 unit
 * cells per axis.  Errors: GMG_E_INVAL. */
int gmg_mesh_create(int dim, int n_coarse, const int32_t* origins, gmg_mesh* out);
/* Refine the flagged leaves (flags[n_leaves], canonical order, nonzero =
 * refine), then close the mesh to 2:1 balance: any two leaves whose closures
 * touch differ by at most one level (this is the paper's complete layer of
 * level l-1 cells around the level-l cells).  Writes the new leaf count. */
int gmg_mesh_refine(gmg_mesh m, const uint8_t* flags, int64_t* n_leaves_after);
int gmg_mesh_num_leaves(gmg_mesh m, int64_t* n);
/* Leaves in canonical order: level[n], anchor[n*dim] (global, units 2^-20). */
int gmg_mesh_leaves(gmg_mesh m, int8_t* level, int64_t* anchor);
int gmg_mesh_dim(gmg_mesh m, int* dim);
int gmg_mesh_destroy(gmg_mesh m);

/* ---------------------------------------------------------------- problem
 * Host setup: leaf DoF numbering with hanging-node constraints (Sec. 2.3),
 * level DoFs with the S/I/D splitting (Sec. 2.3, Fig. 1), copy map from the
 * leaf vector into the level vectors, transfer (family) maps (Sec. 2.2).
 * cell_coeff: [n_leaves] a_K > 0 in canonical leaf order, or NULL for 1.
 * The mesh is only read; it may be destroyed afterwards. */
int gmg_problem_create(gmg_mesh m, const gmg_options* opts, const double* cell_coeff,
                       gmg_problem* out);

/* New problem with the host set-up of `src` (same mesh, degree and
 * coefficient) and other options (precision, smoother, tolerances); the
 * degree must match.  Not bound. */
int gmg_problem_clone(gmg_problem src, const gmg_options* opts, gmg_problem* out);

typedef struct {
  int32_t dim, degree, n_levels, mg_precision;
  int64_t n_dofs;        /* leaf DoFs incl. Dirichlet nodes, excl. hanging nodes */
  int64_t n_hanging;
  int64_t n_leaves;
  int64_t n_free;        /* non-Dirichlet leaf DoFs */
  int64_t level_dofs[24];
  int64_t level_cells[24];
  double lambda_max[24]; /* eigenvalue estimates, valid after gmg_problem_bind (Chebyshev smoother) */
  size_t workspace_bytes;
} gmg_info;
int gmg_problem_info(gmg_problem p, gmg_info* out);

/* Library-owned host arrays for bit-exact checks (valid until destroy).
 * which / element type / length:
 *   GMG_ARR_LEAF_CELLMAP  int32  n_leaves*(k+1)^d  DoF id, or -(h+1) for hanging node h
 *   GMG_ARR_LEAF_DIRICHLET uint8 n_dofs            1 = Dirichlet node
 *   GMG_ARR_CON_OFFSETS   int64  n_hanging+1       CSR offsets of the constraints
 *   GMG_ARR_CON_MASTERS   int32  nnz              master DoF ids, z-major order
 *   GMG_ARR_CON_WEIGHTS   double nnz              coarse basis at the hanging node
 *   GMG_ARR_COPY_LEVEL    int8   n_dofs            level holding leaf DoF i as S or D
 *   GMG_ARR_COPY_INDEX    int32  n_dofs            its index on that level
 *   GMG_ARR_LEVEL_CELLMAP int32  level_cells*(k+1)^d (level given)
 *   GMG_ARR_LEVEL_FLAGS   uint8  level_dofs        0 S, 1 I, 2 D
 *   GMG_ARR_LEVEL_PARENT  int32  level_cells/2^d   parent index in level-1 cells
 *   GMG_ARR_LEAF_CELLMAP_PARENT int32 n_leaves*(k+1)^d  in-cell constraint form: on a face or
 *                         edge shared with a coarser leaf, the DoF of the parent's node at the
 *                         same local position (interpolated in the cell by the 1D embedding)
 *   GMG_ARR_LEAF_MASK     uint16 n_leaves         bits 0-2 child position, 3-5 hanging face
 *                         normal to x/y/z, 6-8 hanging edge along x/y/z
 *   GMG_ARR_LEVEL_PERM    int32  level_dofs        device index of each level DoF (level given):
 *                         levels >= 1 store their vectors in the entity layout of their sibling
 *                         families (interiors, then facets, edges, vertices of the family
 *                         lattice); level 0 keeps its numbering */
enum {
  GMG_ARR_LEAF_CELLMAP = 1,
  GMG_ARR_LEAF_DIRICHLET = 2,
  GMG_ARR_CON_OFFSETS = 3,
  GMG_ARR_CON_MASTERS = 4,
  GMG_ARR_CON_WEIGHTS = 5,
  GMG_ARR_COPY_LEVEL = 6,
  GMG_ARR_COPY_INDEX = 7,
  GMG_ARR_LEVEL_CELLMAP = 8,
  GMG_ARR_LEVEL_FLAGS = 9,
  GMG_ARR_LEVEL_PARENT = 10,
  GMG_ARR_LEAF_CELLMAP_PARENT = 11,
  GMG_ARR_LEAF_MASK = 12,
  GMG_ARR_LEVEL_PERM = 13
};
int gmg_problem_array(gmg_problem p, int which, int level, const void** ptr, int64_t* count);

/* Device memory the problem needs (maps, level and CG vectors, coarse
 * inverse).  The caller allocates it (any HIP device allocation, e.g. a torch
 * uint8 tensor) and keeps it alive until gmg_problem_destroy. */
int gmg_problem_workspace_bytes(gmg_problem p, size_t* bytes);
/* Upload maps into d_workspace and run the device setup on `stream`: Jacobi
 * diagonals, lambda_max estimates (FP64 Lanczos from CG, Sec. 4.1), exact
 * coarse inverse (FP64).  Synchronises the stream.  d_workspace must be
 * 256-byte aligned.  Errors: GMG_E_INVAL (too small), GMG_E_HIP. */
int gmg_problem_bind(gmg_problem p, void* d_workspace, size_t bytes, hipStream_t stream);
int gmg_problem_destroy(gmg_problem p);

/* ---------------------------------------------------------------- solve */

/* Load vector b = C^T M C f (Sec. 2.1 right-hand side with the nodal
 * interpolant; C eliminates hanging nodes), Dirichlet rows zero.
 * d_f: [n_dofs] nodal values (FP64); d_b: [n_dofs]. */
int gmg_rhs(gmg_problem p, const double* d_f, double* d_b, hipStream_t stream);

/* CG with one V-cycle as preconditioner, x0 = 0, until
 * ||r||_2 <= rtol ||b||_2 (Sec. 4.1/4.3).  d_f: nodal right-hand side
 * [n_dofs] (FP64, device); NULL means f = 1.  d_u: [n_dofs] solution.
 * iterations: CG iterations done.  history (host, may be NULL):
 * [max_iter+1] relative residual norms, entry 0 = 1.  Returns GMG_OK,
 * GMG_NOT_CONVERGED, GMG_E_NAN (non-finite residual) or GMG_E_BREAKDOWN
 * (p.Ap <= 0 or r.z <= 0).  Synchronises the stream. */
int gmg_solve(gmg_problem p, const double* d_f, double* d_u, int32_t* iterations,
              double* history, hipStream_t stream);
/* Same as gmg_solve with a precomputed load vector d_b. */
int gmg_solve_rhs(gmg_problem p, const double* d_b, double* d_u, int32_t* iterations,
                  double* history, hipStream_t stream);

/* Test hooks (stream-ordered, no synchronisation):
 * leaf operator q = C^T A C p with Dirichlet rows zeroed (FP64, [n_dofs]);
 * level operator on level l (element type = mg precision, [level_dofs[l]],
 * vectors in the device layout of the level, see GMG_ARR_LEVEL_PERM):
 *   variant 0 (smoother): y = A_l x over all level cells, every row written
 *     (rows of S nodes give A^S x^S when x is zero on I and D nodes);
 *   variant 1 (edge): y^S = A^{SI} x^I: input restricted to I nodes, output
 *     to S rows, other rows 0;
 *   variant 2 (timing): one Chebyshev smoothing step (Sec. 4.1) on the
 *     level's V-cycle work vectors, levels >= 1; d_in and d_out unused;
 * one V-cycle z = B r (FP64 in and out, [n_dofs]). */
int gmg_apply_leaf(gmg_problem p, const double* d_in, double* d_out, hipStream_t stream);
int gmg_apply_level(gmg_problem p, int level, int variant, const void* d_in, void* d_out,
                    hipStream_t stream);
int gmg_vcycle(gmg_problem p, const double* d_r, double* d_z, hipStream_t stream);

/* One V-cycle z_i = B_i r_i (as gmg_vcycle) for each of n bound problems of
 * the same dimension, degree, precision and smoother (several resident
 * solves, Sec. 2.3 local smoothing per problem), with the level sweeps of
 * all of them in one launch each: every smoothing step, residual pass and
 * second restriction pass on level l is one launch over the level-l
 * families of all problems that have a level l (levels aligned from the
 * coarse end); transfers, copies and coarse solves run per problem on the
 * same stream.  Each z_i equals gmg_vcycle's bit for bit.
 * ps: [n] problems (host array); d_r, d_z: [n] device pointers (host
 * arrays), each [n_dofs of its problem].  d_table: device memory the
 * library writes the launch tables to (256-byte aligned, caller-owned);
 * *table_bytes: its size on entry; on return the size needed.  With d_table
 * NULL only the size is returned and nothing is enqueued.  Synchronises the
 * stream before returning.  Errors: GMG_E_INVAL (mixed problems, table too
 * small), GMG_E_STATE (a problem not bound), GMG_E_HIP. */
int gmg_vcycle_batch(const gmg_problem* ps, int n, const double* const* d_r, double* const* d_z, void* d_table,
                     size_t* table_bytes, hipStream_t stream);

/* ------------------------------------------------------ adaptive loop
 * Residual error estimator of the adaptive loop (Sec. 4.3), per leaf K in
 * canonical leaf order:
 *   eta_K = h_K^2 || f_h + a_K Laplace u_h ||_K^2
 *         + sum over the faces F of K of h_K || [a grad u_h . n] ||_F^2,
 * u_h, f_h the cell polynomials of the constrained nodal values of d_u and
 * d_f_nodal (leaf DoF vectors [n_dofs], device), a the problem's cell
 * coefficient; (k+1)-point Gauss quadrature per direction; no term on the
 * domain boundary; a face shared with finer leaves is integrated over each
 * of their faces; h_K the side of K.  d_eta: [n_leaves] device.  The work
 * memory is a caller-owned device workspace (256-byte aligned) of
 * gmg_estimator_workspace_bytes bytes; it receives the problem's face and
 * constraint tables on the first call with that workspace (again after
 * another problem used it).  Errors: GMG_E_INVAL (null argument, workspace
 * too small or misaligned), GMG_E_HIP. */
int gmg_estimator_workspace_bytes(gmg_problem p, size_t* bytes);
int gmg_estimate(gmg_problem p, const double* d_u, const double* d_f_nodal, void* d_ws, size_t ws_bytes,
                 double* d_eta, hipStream_t stream);
/* Marking (Sec. 4.3: the 14.2 % of the leaves with the largest estimates):
 * d_flags[K] = 1 for the round(fraction n_leaves) leaves with the largest
 * d_eta, equal values taken in leaf order, else 0 ([n_leaves] uint8, device;
 * the flags of gmg_mesh_refine once copied to the host).  Same workspace as
 * gmg_estimate.  Errors: GMG_E_INVAL (fraction outside [0, 1]). */
int gmg_mark(gmg_problem p, const double* d_eta, double fraction, uint8_t* d_flags, void* d_ws, size_t ws_bytes,
             hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * V-cycle as gmg_vcycle, with its work memory (level vectors x, g, t, d,
 * operator slots, restricted family values) in a fixed device array of the
 * library, GMG_NOALLOC_SCRATCH_BYTES per GPU, created when the library's
 * code is loaded on a GPU and held until the process ends.  The call
 * allocates nothing (no hipMalloc/hipFree, no allocating library routine);
 * the problem must be bound, with the current device the one it was bound
 * on.  The array starts every call cleared (a fill kernel on `stream`), so
 * the result equals gmg_vcycle's.  All calls on one GPU share the array:
 * calls that overlap on one GPU (other streams, other threads) race and give
 * wrong results; serialise them.  Errors: GMG_E_INVAL when the problem's
 * work memory exceeds GMG_NOALLOC_SCRATCH_BYTES (the message gives the size
 * needed), GMG_E_STATE (not bound, other device), GMG_E_HIP. */
#define GMG_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int gmg_vcycle_noalloc(gmg_problem p, const double* d_r, double* d_z, hipStream_t stream);

/* Seconds of device time of the last gmg_solve* on this problem (events on
 * the caller's stream): [0] whole solve, [1] sum of V-cycles, [2] number of
 * V-cycles. */
int gmg_problem_last_timing(gmg_problem p, double* out3);

/* ---------------------------------------------------------------- serving
 * A request loop for many solves on different adaptive meshes (continuous
 * batching): host threads build each request's maps as it arrives; a
 * scheduler thread admits ready requests in arrival order whenever a slot
 * and enough arena memory are free (first fit), sets them up on the device
 * on the slot's stream and then advances every resident solve one CG
 * iteration per tick.  The requests due in a tick that share dimension,
 * degree, precision, Chebyshev degree and smoother run that iteration as
 * one batched iteration on a batch stream (V-cycle as gmg_vcycle_batch, and
 * the rest of the CG iteration likewise: one launch per step for all of
 * them).  A request alone in its group replays its V-cycle as a captured
 * HIP graph on its own stream.  A finished request frees its slot and memory for
 * the next one.  Results do not depend on the other resident requests (all
 * kernels are deterministic and a batched V-cycle equals the request's own
 * bit for bit). */

typedef struct {       /* seconds on the server clock (0 = gmg_server_create) */
  double arrival;      /* submit */
  double setup_done;   /* host maps built */
  double admitted;     /* slot and memory granted */
  double bound;        /* device set-up done, CG started */
  double finished;     /* solution copied back (or failure) */
} gmg_timing;

typedef struct {
  int64_t queued, running, completed, failed;
  size_t arena_used, arena_peak, arena_bytes;
  double dofs_done;    /* sum of DoFs of completed requests */
  double clock;        /* server clock now */
  int64_t iterations;  /* CG iterations enqueued */
  int64_t batched_iterations;  /* of which with a batched V-cycle */
  int64_t batches;     /* batched V-cycles */
} gmg_server_stats_t;

enum { GMG_REQ_QUEUED = 0, GMG_REQ_SETUP = 1, GMG_REQ_READY = 2, GMG_REQ_BINDING = 3, GMG_REQ_RUNNING = 4,
       GMG_REQ_DONE = 5, GMG_REQ_FAILED = 6, GMG_REQ_WAIT_RHS = 7 };

/* n_f value of gmg_server_submit: the right-hand side follows later through
 * gmg_server_set_rhs */
#define GMG_RHS_LATER ((int64_t)-1)

/* d_arena: device memory owned by the caller (256-byte aligned) that holds
 * the workspaces of resident requests and, at its front, the launch tables
 * of the batched V-cycles (1/32 of it, at most 16 MiB; none, and so no
 * batching, below 2 MiB); arena_bytes is the HBM budget.
 * max_slots: resident requests at most (1..64); host_threads: workers for
 * host set-up and device binding (1..64).  Uses the current device. */
int gmg_server_create(void* d_arena, size_t arena_bytes, int32_t max_slots, int32_t host_threads,
                      gmg_server* out);
/* Queue a solve (the problem of Sec. 2.1 on the request's own mesh).  The
 * server takes the mesh (the handle is invalid afterwards).  cell_coeff:
 * [n_leaves] or NULL for 1 (copied).  Right-hand side, the nodal values f_h
 * (Sec. 2.1 load vector b = C^T M C f_h, as gmg_solve), one of:
 *   f_nodal_host = [n_f] values in canonical leaf DoF order (copied); the
 *     request fails with GMG_E_INVAL when its DoF count differs from n_f;
 *   f_nodal_host = NULL, n_f = 0: f = 1;
 *   f_nodal_host = NULL, n_f = GMG_RHS_LATER: the caller supplies it with
 *     gmg_server_set_rhs once gmg_server_request_dofs reports the DoF count
 *     (the request waits in state GMG_REQ_WAIT_RHS after its host set-up,
 *     without holding a slot or arena memory).
 * A request larger than the arena fails with GMG_E_BUDGET. */
int gmg_server_submit(gmg_server s, gmg_mesh mesh, const gmg_options* opts, const double* cell_coeff,
                      const double* f_nodal_host, int64_t n_f, uint64_t* request_id);
/* DoF count of a request whose host set-up is done (GMG_E_STATE before). */
int gmg_server_request_dofs(gmg_server s, uint64_t request_id, int64_t* n_dofs);
/* Nodal right-hand side of a request submitted with GMG_RHS_LATER: [n_f]
 * values in canonical leaf DoF order (copied).  GMG_E_STATE if the request
 * takes none or already has one; GMG_E_INVAL if n_f differs from its DoF
 * count (when known; otherwise the request fails after its host set-up). */
int gmg_server_set_rhs(gmg_server s, uint64_t request_id, const double* f_nodal_host, int64_t n_f);
int gmg_server_poll(gmg_server s, uint64_t request_id, int32_t* state, int32_t* status);
/* Block until the request is done or failed; GMG_E_STATE on timeout. */
int gmg_server_wait(gmg_server s, uint64_t request_id, double timeout_s);
/* Outputs of a finished request: u_host [n_dofs] (may be NULL; query n_dofs
 * first with u_host = NULL), iterations, history [iterations+1], timing.
 * Returns the solve status, or the failure code of a failed request. */
int gmg_server_result(gmg_server s, uint64_t request_id, double* u_host, int64_t* n_dofs,
                      int32_t* iterations, double* history, gmg_timing* timing);
/* Forget a finished request. */
int gmg_server_release(gmg_server s, uint64_t request_id);
int gmg_server_stats(gmg_server s, gmg_server_stats_t* out);
/* Batched V-cycles on (enable = 1, the default) or off (every request
 * replays its own V-cycle graph); results are the same either way. */
int gmg_server_set_batching(gmg_server s, int enable);
/* hold = 1: resident solves are not advanced (admission and set-up go on),
 * so that requests arriving in a burst start their iterations together, or
 * to quiesce the device; hold = 0 resumes. */
int gmg_server_hold(gmg_server s, int hold);
/* Stops the threads after the current tick; resident solves are abandoned. */
int gmg_server_destroy(gmg_server s);

#ifdef __cplusplus
}
#endif
#endif
