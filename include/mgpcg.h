/*
 * mgpcg.h - C ABI of the MI355X (gfx950) global-local multigrid library.
 *
 * The library solves the reduced finite-element Poisson system A u = b of
 * continuous Lagrange P1/P2 (2D, 3D) or P3 (2D) elements on a simplicial mesh
 * (Chen & Wells, arXiv 2402.12947, Sec. 2, eq. system_finest; Sec. 6.1) with
 * conjugate gradients preconditioned by one non-nested geometric Galerkin
 * multigrid V-cycle per iteration (Algorithm alg:mg; Sec. 6.2).  The smoother
 * is the global-local combined smoother of Sec. 4.2: a local residual
 * correction S_c (exact dense solves on patches around cells whose normalised
 * radius ratio is below a threshold, Sec. 4.1, Sec. 4.4), a Jacobi-
 * preconditioned Chebyshev sweep S_g over the whole level with the adjusted
 * largest eigenvalue of Sec. 5, then S_c again.
 *
 * Conventions shared by every entry point
 *  - Meshes are host arrays owned by the caller; mg_setup copies what it
 *    needs and keeps no caller pointer.  Cells must be positively oriented.
 *  - Homogeneous Dirichlet conditions (u = 0) are imposed on the DOFs of
 *    boundary facets whose vertices are all flagged in dirichlet_vertex; the
 *    rest of the boundary carries the natural (zero-flux) condition.
 *  - DOF numbering: vertex DOFs first (id = vertex id), then edge DOFs in the
 *    order of the sorted (low vertex, high vertex) pairs (P3: two per edge,
 *    the node nearer the low vertex first), then P3 cell interiors in cell
 *    order.  Solver vectors (b, u, f) hold the FREE (non-Dirichlet) DOFs of
 *    level 0 in that order; their length is mg_level_info.n_free.
 *  - Vectors passed to mg_smooth / mg_vcycle / mg_pcg_solve / mg_rhs_from_nodal
 *    are DEVICE pointers to FP64 arrays, accessed on the context's stream.
 *  - Errors: a negative status; mg_last_error(ctx) (or mg_global_error() when
 *    mg_setup failed and returned no context) holds a message.  A positive
 *    status is a warning with valid outputs.  Outputs are undefined after an
 *    error.  A context is not thread-safe; distinct contexts are independent.
 */
#ifndef MGPCG_H
#define MGPCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MG_API_VERSION 1
#define MG_MAX_HISTORY 1024

typedef struct mg_ctx mg_ctx;

typedef enum {
  MG_OK = 0,
  MG_NOT_CONVERGED = 1,   /* maxit reached; u holds the last iterate          */
  MG_ERR_ARG = -1,        /* bad argument (NULL, size, aliasing, option)        */
  MG_ERR_MESH = -2,       /* index out of range or non-positive cell volume     */
  MG_ERR_LOCATE = -3,     /* a fine DOF node lies outside the next coarser mesh */
  MG_ERR_NOT_SPD = -4,    /* non-positive pivot / diagonal: system not SPD      */
  MG_ERR_BREAKDOWN = -5,  /* CG breakdown: p.Ap <= 0 or a non-finite value      */
  MG_ERR_HIP = -6,        /* a HIP runtime call failed                          */
  MG_ERR_OOM = -7,        /* device allocation failed                           */
  MG_ERR_LIMIT = -8       /* a documented size limit was exceeded               */
} mg_status;

enum { MG_FP64 = 0, MG_MIXED = 1 };
enum { MG_PATCH_MERGE = 0, MG_PATCH_OVERLAP = 1 };
enum { MG_SMOOTHER_CHEBYSHEV = 0, MG_SMOOTHER_SGS = 1 };
enum { MG_PROBLEM_POISSON = 0, MG_PROBLEM_ELASTICITY = 1 };

/* One level of the hierarchy: an independent simplicial mesh of the domain. */
typedef struct {
  int32_t dim;                      /* 2 or 3                                  */
  int64_t n_vertices;
  const double *coords;             /* host [n_vertices * dim]                 */
  int64_t n_cells;
  const int32_t *cells;             /* host [n_cells * (dim + 1)], vertex ids  */
  const uint8_t *dirichlet_vertex;  /* host [n_vertices], 1 = on Gamma_D       */
} mg_mesh;

/* Solver options; mg_default_options fills the paper's values. */
typedef struct {
  int32_t degree;           /* Lagrange degree 1, 2 or 3 (3: dim 2 only)       */
  int32_t precision;        /* MG_FP64, or MG_MIXED: FP32 V-cycle (smoothers,
                               transfers, patch solves) inside FP64 CG; the
                               coarsest solve stays FP64                       */
  int32_t nu;               /* smoother applications pre and post (Sec. 6: 2)  */
  int32_t cheb_degree;      /* Chebyshev polynomial degree per S_g (2)         */
  double cheb_lo_frac;      /* lower bound = frac * upper (Sec. 3.2: 0.1)      */
  int32_t local_correction; /* 1: S_c -> S_g -> S_c; 0: S_g only               */
  int32_t adjusted_eig;     /* 1: Chebyshev upper bound = adjusted lambda_max
                               (Sec. 5); 0: lambda_max of D^-1 A               */
  int32_t patch_policy;     /* MG_PATCH_MERGE (disjoint subdomains, one colour)
                               or MG_PATCH_OVERLAP (coloured, sequential)     */
  double eig_tol;           /* Lanczos Ritz-residual tolerance (1e-8)          */
  int32_t eig_maxit;        /* Lanczos step limit (200)                        */
  int32_t use_graph;        /* 1: replay from captured hipGraphs: each CG
                               iteration of the solvers (V-cycle and CG
                               updates, one graph per block width) and the
                               V-cycle of mg_vcycle / mg_vcycle_solve          */
  int32_t sell_sigma;       /* SELL row-sorting window: 0 = autotune, 1 = off,
                               else a multiple of 64                          */
  void *stream;             /* hipStream_t to run on; NULL = library-owned     */
  int32_t global_smoother;  /* S_g: MG_SMOOTHER_CHEBYSHEV (Chebyshev-Jacobi,
                               the default) or MG_SMOOTHER_SGS: one forward and
                               one backward multicolour Gauss-Seidel sweep
                               (Sec. 3.2, Sec. 6.1); the rows are coloured
                               greedily in canonical order, each row taking the
                               smallest colour unused by its lower-numbered
                               neighbours; no eigenvalue estimate is made      */
  int32_t problem;          /* MG_PROBLEM_POISSON: -lap u = f (Sec. 6.1), or
                               MG_PROBLEM_ELASTICITY: -div sigma(u) = f with
                               sigma = 2 mu eps(u) + lambda tr(eps(u)) I
                               (Sec. 6.2), vector Lagrange elements, unknown
                               (scalar DOF s, component c) = s * dim + c, all
                               components of a Dirichlet DOF clamped          */
  double young;             /* E (elasticity; paper: 6.9e10)                   */
  double poisson_ratio;     /* nu (elasticity; paper: 0.33), 0 <= nu < 0.5     */
  int32_t sell_unroll;      /* gathers in flight per lane in the sparse
                               products: 0 = chosen per level by timing, 4, 8 */
  int32_t sell_mask;        /* -1 = chosen per matrix by timing; 1 = skip the
                               values of each row's padding past the shortest
                               row of its slice; 0 = read every stored entry.
                               The result is the same bitwise either way      */
  int32_t sell_rpl;         /* lanes per row of the level operators' sparse
                               products: 0 = chosen per level by timing,
                               1, 2, 4, 8, 16 or 32 (the transfer operators
                               take at most 8)                                 */
  int32_t patch_fused;      /* 1: a colour whose patches fit the level's
                               one-workgroup class (patch_small_bound) and do
                               not couple to each other runs its local
                               correction as one launch, a coupled colour as
                               two; 0: always three launches (the same result
                               bitwise where a tile row fits one chunk)       */
  int32_t use_initial_guess; /* 0: the solvers (mg_pcg_solve and its block and
                               batch forms, mg_vcycle_solve) start from u = 0
                               and ignore u on entry; 1: they start from the u
                               passed in (a warm start)                       */
  int32_t sell_colform;     /* column indices of the sparse layouts: 0 = per
                               slice the narrowest form that fits (16-bit in
                               two windows of 32768, in eight of 8192, in
                               sixteen of 4096, else 32-bit); 1 = start at the
                               eight-window form, 2 = at the sixteen-window
                               form, 3 = 32-bit everywhere (same results; for
                               testing every decode path)                     */
  int32_t patch_factor_f32; /* MG_MIXED only.  1: factor the patch systems on
                               the FP32 matrix cores (FP32 accumulate) after
                               a symmetric diagonal equilibration, and keep
                               the FP64 factorisation for the patches whose
                               scaled pivots fall below 2^-12 (or that hold
                               more than 2048 DOFs); 0: factor every patch in
                               FP64.  The inverse is stored in FP32 either
                               way                                             */
  int32_t patch_refine;     /* 1: every patch solve takes one step of
                               iterative refinement, e = X r, then
                               e += X (r - A^[d] e) with the residual of the
                               patch system formed in FP64 (X the stored
                               inverse; costs a second product with X and the
                               patch rows once more); 0: e = X r             */
  int32_t patch_inherit_levels; /* 0 (the paper): each level's patches come
                               from its own cells' quality.  k > 0: levels
                               1..k (not the coarsest) also take the patches
                               inherited through the interpolation from the
                               finest level's degraded cells: seeds = the free
                               DOFs of each degraded cell of level 0; level
                               l+1 inherits, per seed, the coarse DOFs that
                               P_l couples to it (the free DOFs of the coarse
                               cells containing its nodes); the connected
                               components of these sets (shared DOFs, ordered
                               by smallest DOF) follow the level's own patches
                               (MERGE: merged with the own patches they share
                               DOFs with; OVERLAP: coloured).  The Galerkin
                               operator A_(l+1) = P^T A_l P carries the
                               degraded cells' stiffness into exactly those
                               rows                                            */
  int32_t patch_chunk;      /* tiles per row item of the packed patch and
                               coarsest inverses: 0 = chosen per level by
                               timing (16, 8 or 32), else 8, 16 or 32        */
  int32_t patch_small_bound; /* one-workgroup local correction (patches of up
                               to this many DOFs in one launch per colour):
                               0 = size class chosen per level by timing among
                               128, 256 and 384 (and the three-launch path),
                               128, 256 or 384 = that class where every patch
                               fits it, -1 = always the three-launch path.
                               Needs patch_fused = 1 and patch_refine = 0     */
  int32_t coarse_solver;    /* coarsest-level direct solve: 0 = nested
                               dissection from 12288 unknowns, the dense
                               explicit inverse below; 1 = dense inverse;
                               2 = nested dissection                          */
  int32_t coarse_nd_leaf;   /* largest leaf of the nested dissection (1024)    */
  int32_t sell_layout_levels; /* number of levels that sell_layout covers      */
  const int32_t *sell_layout; /* NULL, or host [4 * sell_layout_levels]: for
                               level l the values (sigma, unroll, mask, rpl)
                               that fix that level operator's layout as
                               sell_sigma, sell_unroll, sell_mask and sell_rpl
                               do for every level (0, 0, -1, 0 leave the choice
                               to the autotuner); copied by mg_setup.  Lets a
                               measurement repeat the layouts of an earlier
                               run, whose choices mg_level_info reports      */
  int32_t patch_rows_rpl;   /* lanes per row of the patch-row residual (the
                               rows of A at the patch DOFs): 0 = chosen per
                               level by timing, else 1, 2, 4 or 8 (1 with
                               patch_refine)                                   */
} mg_options;

typedef struct {
  int32_t iterations;       /* number of products with A (Sec. 6 stopping)     */
  int32_t converged;
  double rel_residual;      /* ||r||/||b|| of the recursively updated residual */
  double true_rel_residual; /* ||b - A u||/||b|| recomputed at exit, FP64      */
  double solve_ms;          /* wall time of the solve on the stream            */
  int32_t n_history;
  double history[MG_MAX_HISTORY]; /* rel. residual after each iteration, [0]=1 */
} mg_solve_stats;

typedef struct {
  int64_t n_vertices, n_cells;
  int64_t n_dofs;           /* all DOFs of the level's mesh                    */
  int64_t n_free;           /* unknowns of the level's operator                */
  int64_t nnz;              /* nonzeros of A_l (CSR)                           */
  int64_t n_flagged;        /* cells with gamma < threshold                    */
  int32_t n_patches, n_colours, max_patch;
  int64_t sum_patch_dofs;
  double gamma_min;
  double lambda_max;        /* lambda_max(D^-1 A_l) (Lanczos)                  */
  double lambda_adj;        /* adjusted lambda_max (Sec. 5)                    */
  double cheb_lo, cheb_hi;  /* Chebyshev interval used                         */
  int32_t lanczos_steps, lanczos_steps_adj;
  int32_t sell_sigma;       /* SELL sorting window chosen                      */
  int64_t sell_stored;      /* stored SELL entries incl. padding               */
  int32_t is_coarsest;
  double setup_ms;          /* setup time spent on this level                  */
  int64_t sell_nnz16;       /* nonzeros stored with 16-bit column indices      */
  int32_t n_components;     /* unknowns per DOF node (1; dim for elasticity):
                               n_free = n_components * free DOF nodes          */
  int32_t sell_unroll;      /* gathers in flight per lane in the level's
                               sparse products (4 or 8, chosen by timing)      */
  int32_t sell_mask;        /* 1: the level's sparse products skip the values
                               of each row's padding past the shortest row of
                               its slice; 0: they read every stored entry
                               (same result bitwise; chosen by timing)         */
  int32_t sell_rpl;         /* lanes per row of the level's operator products
                               (1, 2, 4, 8, 16 or 32; chosen by timing)       */
  int32_t patch_fused_colours; /* patch colours whose local correction runs
                               as one launch                                   */
  int64_t sell_slices;      /* slices of the level operator's SELL layout      */
  int64_t sell_slices_multiwindow; /* of them with 16-bit columns in 8 or 16
                               windows (decoded with a cross-lane read)        */
  int64_t sell_slices_32bit; /* of them with 32-bit columns                    */
  int64_t sell_slices_16window; /* of the multiwindow slices, those with 16   */
  int32_t patches_f32;      /* patches factored on the FP32 matrix cores       */
  int32_t patches_inherited; /* inherited components (patch_inherit_levels)   */
  int32_t patch_small_bound; /* one-workgroup class used (128, 256, 384), 0 =
                               the three-launch path                          */
  int32_t patch_chunk;      /* tiles per row item of the level's packed
                               inverses (patches; the coarsest level: its
                               inverse)                                        */
  int32_t coarse_nd_supernodes; /* coarsest level: supernodes of the nested
                               dissection (0: dense inverse)                  */
  double coarse_solve_bytes; /* coarsest level: FP64 matrix bytes one solve
                               reads (dense: packed lower tiles; dissection:
                               diagonal-block inverses and the tile rows of L
                               below them, forward and backward)              */
  int32_t patch_rows_rpl;   /* lanes per row of the patch-row residual         */
} mg_level_info;

/* Arrays that mg_get_array copies to a caller-owned HOST buffer. */
enum {
  MG_ARR_QUALITY = 1,      /* double  [n_cells]  normalised radius ratio        */
  MG_ARR_FLAGS = 2,        /* uint8   [n_cells]  gamma < threshold              */
  MG_ARR_PATCH_PTR = 3,    /* int32   [n_patches + 1]                           */
  MG_ARR_PATCH_DOFS = 4,   /* int32   [sum_patch_dofs] free DOF ids, ascending  */
  MG_ARR_PATCH_COLOUR = 5, /* int32   [n_patches]                               */
  MG_ARR_LOCATE = 6,       /* int32   [n_free] coarse cell of each free DOF node
                              (levels above the coarsest)                     */
  MG_ARR_FREE_DOFS = 7,    /* int32   [n_free / n_components] canonical DOF id
                              of each free DOF node (LOCATE likewise)        */
  MG_ARR_DOF_NODES = 8,    /* double  [n_dofs * dim] node coordinates          */
  MG_ARR_A_ROWPTR = 9,     /* int64   [n_free + 1]                              */
  MG_ARR_A_COLS = 10,      /* int32   [nnz]                                     */
  MG_ARR_A_VALS = 11,      /* double  [nnz]                                     */
  MG_ARR_P_COLS = 12,      /* int32   [n_free * width] (row-major, -1 = none)   */
  MG_ARR_P_VALS = 13,      /* double  [n_free * width]                          */
  MG_ARR_CELL_DOFS = 14,   /* int32   [n_cells * n_local] canonical DOF ids     */
  MG_ARR_P_WIDTH = 15,     /* int32   [1] coarse DOFs per cell (ELL width)      */
  MG_ARR_SGS_COLOUR = 16   /* int32   [n_free] Gauss-Seidel colour of each
                              unknown (MG_SMOOTHER_SGS, levels above the
                              coarsest)                                       */
};

/* Fills *opt with: degree 1, MG_FP64, nu 2, cheb_degree 2, cheb_lo_frac 0.1,
 * local_correction 1, adjusted_eig 1, MG_PATCH_MERGE, eig_tol 1e-8,
 * eig_maxit 200, use_graph 0, sell_sigma 0, stream NULL,
 * global_smoother MG_SMOOTHER_CHEBYSHEV, problem MG_PROBLEM_POISSON,
 * young 6.9e10, poisson_ratio 0.33, sell_unroll 0, sell_mask -1, sell_rpl 0,
 * patch_fused 1, use_initial_guess 0, sell_colform 0, patch_factor_f32 1,
 * patch_refine 0, patch_inherit_levels 0, patch_chunk 0, patch_small_bound 0,
 * coarse_solver 0, coarse_nd_leaf 1024, sell_layout_levels 0, sell_layout NULL,
 * patch_rows_rpl 0. */
void mg_default_options(mg_options *opt);

/* Builds the hierarchy (Sec. 2; Sec. 4.4; Sec. 5): per level the DOF map,
 * cell quality gamma (Sec. 3 eq. radius_ratio, read as d R_I / R_C), the
 * local-correction patches (cells with gamma < quality_threshold grown by
 * patch_layers vertex layers), the fine-level assembly, the interpolation
 * prolongation by point location and the Galerkin operators
 * A_(l+1) = P_l^T A_l P_l, the patch factorisations, the (adjusted) largest
 * eigenvalues and, on the coarsest level, a dense Cholesky factorisation.
 * levels[0] is the finest mesh.  On success *out owns all device memory it
 * allocated until mg_destroy.  On failure *out = NULL and nothing leaks.
 * Limits: a local-correction patch of more than 16384 DOFs, a coarsest level
 * of more than 60000 unknowns or a Galerkin row of more than 3072 nonzeros
 * fail with MG_ERR_LIMIT.  With MG_SETUP_LOG=1 in the environment every
 * finished setup phase is reported on stderr.
 * Errors: MG_ERR_ARG, MG_ERR_MESH, MG_ERR_LOCATE, MG_ERR_NOT_SPD, MG_ERR_HIP,
 * MG_ERR_OOM, MG_ERR_LIMIT. */
mg_status mg_setup(const mg_mesh *levels, int32_t n_levels, double quality_threshold,
                   int32_t patch_layers, const mg_options *opt, mg_ctx **out);

/* u <- S^nu(A_l, b, u) (Sec. 2 smoother notation): nu applications of the
 * combined smoother S_c -> S_g -> S_c (Sec. 4.2) on level `level`, in the
 * context's precision.  b, u: device FP64 vectors of the level's n_free;
 * b must not alias u.  Not available on the coarsest level. */
mg_status mg_smooth(mg_ctx *c, int32_t level, const double *b, double *u, int32_t nu);

/* u <- Vcycle(A_0, b, u) (Algorithm alg:mg) on level 0 from the given u. */
mg_status mg_vcycle(mg_ctx *c, const double *b, double *u);

/* Allocation-free form of mg_vcycle, for callers that cannot allocate device
 * memory: code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc.  It computes the same cycle as mg_vcycle (bitwise the same
 * u) but keeps its four level-0 staging vectors (b and u in the solve order,
 * the residual, the correction) in one static device array of the library,
 * MG_NOALLOC_SCRATCH_BYTES per GPU, created when the library is loaded and
 * held until the process ends; it calls no allocating routine and does not
 * synchronise: the cycle is enqueued on the context's stream and u is valid
 * once that stream has run it.  The cycle runs eagerly (no captured graph)
 * and without kernel timing.  Limit: n_free(0) <= MG_NOALLOC_MAX_UNKNOWNS,
 * else MG_ERR_LIMIT.  Every call on one GPU shares that GPU's array, which
 * keeps the last call's contents (nothing in it needs to start at zero: every
 * entry a call reads was written earlier in the same call): calls ordered on
 * one stream are safe, calls that overlap in time on one GPU (contexts on
 * different streams, several host threads) race and give undefined results.
 * b, u: device FP64 vectors of n_free(0); b must not alias u.
 * Errors: MG_ERR_ARG, MG_ERR_LIMIT, MG_ERR_HIP. */
#define MG_NOALLOC_MAX_UNKNOWNS 1048576
#define MG_NOALLOC_SCRATCH_BYTES (4 * 8 * MG_NOALLOC_MAX_UNKNOWNS)
mg_status mg_vcycle_noalloc(mg_ctx *c, const double *b, double *u);

/* CG on A_0 u = b preconditioned by one V-cycle per iteration (Sec. 6.2),
 * from u = 0 (or from the u passed in when use_initial_guess = 1: r_0 =
 * b - A u_0), stopping when ||b - A u||_2 <= rtol ||b||_2 (Sec. 6) on the
 * recursively updated residual; a warm start that already meets the tolerance
 * returns u unchanged after 0 iterations, and b = 0 returns u = 0.  st may be
 * NULL.  Returns MG_NOT_CONVERGED if maxit iterations were not enough (u holds
 * the last iterate), or MG_ERR_BREAKDOWN (p.Ap <= 0, or a non-finite value,
 * one in b included). */
mg_status mg_pcg_solve(mg_ctx *c, const double *b, double *u, double rtol, int32_t maxit,
                       mg_solve_stats *st);

/* Several right-hand sides of one operator (the block form of mg_pcg_solve):
 * solves A_0 u[r] = b[r], r < nrhs, each column with exactly the method,
 * scalars and stopping rule of mg_pcg_solve, but advanced together in blocks
 * of up to 4 columns whose vectors are interleaved, so that every operator
 * stream of the cycle (the smoothers' sparse products, residuals, transfers,
 * patch rows) and of CG is read once per block instead of once per column.
 * A column that has converged keeps its iterate while the others go on.
 * With use_initial_guess = 1 every column starts from its u[r] on entry.
 * b[r], u[r]: device FP64 vectors of n_free(0); no u[r] may alias another
 * vector.  st (may be NULL) receives nrhs records; solve_ms is the time of the
 * block the column ran in.  Results agree with column-by-column mg_pcg_solve
 * to rounding (the order of a few sums differs).  Returns MG_NOT_CONVERGED if
 * any column did not converge in maxit iterations, MG_ERR_BREAKDOWN if one
 * broke down. */
mg_status mg_pcg_solve_multi(mg_ctx *c, int32_t nrhs, const double *const *b, double *const *u, double rtol,
                             int32_t maxit, mg_solve_stats *st);

/* Multigrid as a stationary solver (Sec. 2, Algorithm alg:mg repeated; the
 * Poisson experiments of Sec. 6.1): from u = 0 (or the u passed in when
 * use_initial_guess = 1), u <- Vcycle(A_0, b, u) until
 * ||b - A u||_2 <= rtol ||b||_2 (the residual recomputed after every cycle) or
 * maxit cycles.  st (may be NULL): iterations = cycles, history = relative
 * residual after each cycle.  Returns MG_NOT_CONVERGED if maxit cycles were
 * not enough (u holds the last iterate), MG_ERR_BREAKDOWN on a non-finite
 * residual. */
mg_status mg_vcycle_solve(mg_ctx *c, const double *b, double *u, double rtol, int32_t maxit,
                          mg_solve_stats *st);

/* Many-instance solve (the serving pattern of independent problems): solves
 * the n_inst x nrhs systems A_i u_(i,r) = b_(i,r) of the contexts cs[i] together
 * with the same method and stopping rule as mg_pcg_solve.  b[i * nrhs + r] and
 * u[i * nrhs + r] are device FP64 vectors of instance i's n_free.  One host
 * thread drives every instance: each solves its right-hand sides as the block
 * runs of mg_pcg_solve_multi on its own context stream, and an instance whose
 * last enqueued iteration has completed (polled, no common barrier) is given
 * its next one at once, so the instances' kernels overlap on the GPU; with
 * use_graph = 1 an iteration is one launch of the context's captured CG
 * iteration graph.  The contexts must be distinct.  st (may be NULL) receives
 * n_inst * nrhs records; *wall_ms (may be NULL) the wall time of the whole
 * batch.  An instance that fails stops there while the others go on.
 * Returns the first error of the lowest-numbered failing instance (its
 * message in mg_last_error(cs[i])), else MG_NOT_CONVERGED if any system did
 * not converge, else MG_OK. */
mg_status mg_pcg_solve_batch(mg_ctx *const *cs, int32_t n_inst, int32_t nrhs, const double *const *b,
                             double *const *u, double rtol, int32_t maxit, mg_solve_stats *st,
                             double *wall_ms);

/* b = M f_hat restricted to the free DOFs: the consistent-mass load of nodal
 * data f_hat given at ALL n_dofs DOFs of level 0 (device FP64). */
mg_status mg_rhs_from_nodal(mg_ctx *c, const double *f_nodal, double *b);

mg_status mg_get_level_info(const mg_ctx *c, int32_t level, mg_level_info *out);

/* Copies array `what` (MG_ARR_*) of `level` to the host buffer `out`, which
 * must be large enough (sizes above, from mg_get_level_info). */
mg_status mg_get_array(const mg_ctx *c, int32_t level, int32_t what, void *out);

/* Device-event timing of the solve phase: when enabled (and until disabled),
 * every launch of the full Chebyshev step kernel on each level, and every
 * coarsest solve (the product with the coarsest level's stored inverse or
 * the nested-dissection solve), is bracketed by HIP events on the context's
 * stream, and the V-cycles and CG iterations run eagerly even when
 * use_graph = 1.  mg_level_kernel_time returns, for one
 * level, the number of such launches since enabling and their summed
 * duration in milliseconds (level < coarsest: Chebyshev steps; level =
 * coarsest: coarsest solves); mg_kernel_time is its level-0 form.  Both
 * synchronise the stream.  Enabling again resets the sums. */
mg_status mg_enable_kernel_timing(mg_ctx *c, int32_t enable);
mg_status mg_kernel_time(mg_ctx *c, int64_t *launches, double *total_ms);
mg_status mg_level_kernel_time(mg_ctx *c, int32_t level, int64_t *launches, double *total_ms);

/* Bytes one launch of the level-0 Chebyshev step kernel must move at least:
 * matrix values and column indices once ((v + 2) bytes per entry stored with a
 * 16-bit index, (v + 4) otherwise), x, b and D^-1 read and x' written every
 * step, the direction d written by all steps but the last and read by all but
 * the first, averaged over the k steps: v (4 + 2 (k - 1) / k) bytes per row;
 * v = 8 (FP64) or 4 (FP32 mixed mode). */
mg_status mg_cheb_algorithmic_bytes(const mg_ctx *c, double *bytes);

/* Practical streaming ceilings of the GPU (no context needed): kind 0 = one
 * read stream, 1 = copy (one read, one write stream), 2 = seven read streams
 * and one write stream (the read/write mix of the Chebyshev step).  Moves
 * `bytes` (>= 1 MiB, in device buffers it allocates and frees) `reps` times
 * with 16-byte non-temporal accesses, one pass per element, and returns the
 * achieved rate in GB/s (10^9 bytes/s) in *gbs. */
mg_status mg_stream_probe(int32_t kind, int64_t bytes, int32_t reps, double *gbs);

const char *mg_last_error(const mg_ctx *c);
const char *mg_global_error(void);
void mg_destroy(mg_ctx *c);

#ifdef __cplusplus
}
#endif
#endif /* MGPCG_H */
