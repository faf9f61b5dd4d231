/*
 * bcmg.h -- C ABI of a ghost-point geometric multigrid for the Poisson
 * equation on level-set domains embedded in a uniform Cartesian grid
 * (Coco, Mazza & Semplice, "A ghost-point smoothing strategy for geometric
 * multigrid on curved boundaries", arXiv 2207.14208), built for AMD Instinct
 * MI355X (gfx950).  Every step of the cycle runs as a HIP kernel on the
 * device; the host only validates arguments, sizes buffers and launches.
 *
 * Problem (Sec. 3, eq. mainProblem2D; Sec. 3.3; Sec. 4):
 *   box D = [-1,1]^d, d in {1,2,3}, nodes x_i = -1 + i h, h = 2/N, i = 0..N;
 *   Omega = {phi < 0};  -Laplace(u) = f in Omega;  u = g on the curved
 *   boundary (ghost-point Dirichlet rows, eq. BCh);  u = g_B on nodes of the
 *   box faces inside Omega (eliminated Dirichlet nodes).
 *
 * Node arrays are dense, (N+1)^d entries, x fastest (index i + n j + n^2 k,
 * n = N+1).  Node classes (Sec. 3.3 partition of D_h):
 *   BCMG_OUTSIDE 0  inactive node
 *   BCMG_INSIDE  1  phi < 0, not on a box face: interior unknown
 *   BCMG_GHOST   2  phi >= 0 with an INSIDE axis neighbour: ghost unknown
 *   BCMG_BOXDIR  3  phi < 0 on a box face: fixed value g_B
 *
 * Conventions for every call:
 *   - pointers named *_dev are device pointers (hipMalloc'd or torch CUDA
 *     tensors); *_host are host pointers.  The library never frees caller
 *     memory and never keeps a caller pointer beyond the call, except u_dev
 *     in a batch slot (kept until bcmg_batch_remove).
 *   - calls are ordered on the problem's stream (given at setup).  Calls that
 *     return host values synchronise that stream.
 *   - every call returns a bcmg_status; on failure bcmg_last_error() holds a
 *     thread-local message.  Arguments are validated on the host before any
 *     launch; a failed setup leaves no handle.
 *   - the library is not thread-safe per handle: calls on one problem or
 *     batch must not overlap.
 */
#ifndef BCMG_H
#define BCMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t bcmg_status;
#define BCMG_OK 0
#define BCMG_ERR_INVALID 1       /* bad argument (size, pointer, option, NaN in phi) */
#define BCMG_ERR_OOM 2           /* device allocation failed */
#define BCMG_ERR_DEVICE 3        /* HIP runtime error */
#define BCMG_ERR_NOT_CONVERGED 4 /* max_cycles reached before rel_tol */
#define BCMG_ERR_DIVERGED 5      /* residual non-finite or grew 1e3-fold */
#define BCMG_ERR_STATE 6         /* call not valid in the handle's state */

#define BCMG_OUTSIDE 0
#define BCMG_INSIDE 1
#define BCMG_GHOST 2
#define BCMG_BOXDIR 3

#define BCMG_FP64 0   /* every step in FP64 */
#define BCMG_MIXED 1  /* FP32 cycle on the correction, FP64 residual, update and coarse solve */

/* Dirichlet rows (Neumann rows: dtau / h, with the forms of Prop. optN /
 * opt3DN and G0 = p e^{-p t} over p in [acosh 2, acosh(2d-1)], whose maximum
 * may be interior at p = 1/t) */
#define BCMG_DTAU_OPT_EXP 0  /* dtau = 2/(e^{-p1 t} + e^{-pd t}), Remark exptheta2D */
#define BCMG_DTAU_OPT_POLY 1 /* dtau = 2/(min|G0| + max|G0|), Prop. opt / opt3D, eq. coeff (coeffN) */
#define BCMG_DTAU_CONST 2    /* dtau = dtau_const on every ghost (Neumann: dtau_const * h) */

/* boundary condition B u = g on Gamma (Sec. 3.3; the box faces keep the
 * Dirichlet data g_B) */
#define BCMG_BC_DIRICHLET 0  /* B u = u */
#define BCMG_BC_NEUMANN 1    /* B u = grad u . n, n the ghost's outward unit normal */

#define BCMG_RESTRICT_RENORM_FW 0 /* FW weights renormalised over the admissible nodes */
#define BCMG_RESTRICT_PLAIN_MEAN 1 /* unweighted mean over the admissible nodes */

typedef struct bcmg_problem bcmg_problem;
typedef struct bcmg_batch bcmg_batch;

typedef struct {
    int32_t nu1;           /* pre-smoothing steps (default 2) */
    int32_t nu2;           /* post-smoothing steps (default 1) */
    int32_t coarsest_N;    /* intervals per axis on the coarsest grid (must be 4: 5^d nodes) */
    int32_t max_cycles;    /* cycle limit of a solve (default 100, at most 1000) */
    int32_t precision;     /* BCMG_FP64 or BCMG_MIXED */
    int32_t dtau_mode;     /* BCMG_DTAU_* */
    double dtau_const;     /* used by BCMG_DTAU_CONST */
    int32_t ext_iters;     /* K: Jacobi sweeps of the normal extension (default 4, 1..8) */
    int32_t restrict_mode; /* BCMG_RESTRICT_* */
    int32_t seg_len;       /* row tile: nodes per row segment handled by one wavefront (64 or 128, default 128) */
    int32_t bc;            /* BCMG_BC_* on Gamma (default Dirichlet) */
    double reaction;       /* c >= 0 of c u - Laplace u = f (default 0: Poisson; 1: the reaction-diffusion
                              tests of Sec. 3.3 / Sec. 4.2 with Neumann rows) */
    int32_t layout;        /* BCMG_LAYOUT_*: storage order of the library's own finest-level arrays */
    int32_t cycle;         /* BCMG_CYCLE_V (default) or BCMG_CYCLE_W */
    int32_t smoother;      /* BCMG_SMOOTH_RB (red-black Gauss-Seidel, default) or BCMG_SMOOTH_JACOBI */
    int32_t check_interval; /* bcmg_solve: at most this many cycles per convergence check (1..16, default 1:
                               a check after every cycle); see bcmg_solve */
} bcmg_options;

/* Cycle shape (Sec. 2.1: the two-grid scheme applied recursively, gamma
 * times on each coarse level): V (gamma = 1) or W (gamma = 2 on every level
 * but the one above the coarsest, whose coarse problem is solved exactly
 * once).  A W-cycle runs every level by launches (no per-problem coarse
 * workgroup), and a batch of W-cycle problems needs them all to have the
 * same number of levels. */
#define BCMG_CYCLE_V 0
#define BCMG_CYCLE_W 1
/* Interior smoother of each smoothing step (the ghost relaxation follows
 * either): red-black Gauss-Seidel, or weighted Jacobi (Sec. 2.1: omega D +
 * (1 - omega) I with omega = 2d / (2d + 1), 2/3 in 1D), whose new values go
 * through the level's residual array (two launches).  Weighted Jacobi runs
 * every level but the coarsest by launches and needs a nonsingular coarsest
 * level. */
#define BCMG_SMOOTH_RB 0
#define BCMG_SMOOTH_JACOBI 1

/* Storage order of the FP32 level arrays of a mixed-precision problem (the
 * caller's arrays are always x fastest).  SPLIT (default): on the finest
 * level when it has more than 131072 nodes, and on a coarser level with more
 * than 4194304 nodes, the nodes of even index are stored before those of odd
 * index; with N + 1 odd these are the two colours of the red-black sweep, so
 * each colour pass reads and writes contiguous halves, with 16-byte loads and
 * stores.  NATURAL: x fastest everywhere.  The arithmetic is the same, so
 * both give the same bits. */
#define BCMG_LAYOUT_NATURAL 0
#define BCMG_LAYOUT_SPLIT 1

typedef struct {
    int32_t cycles;        /* V-cycles performed */
    bcmg_status status;    /* BCMG_OK, _NOT_CONVERGED or _DIVERGED */
    double r0;             /* ||r^0||_2 over INSIDE and GHOST rows */
    double r_final;        /* ||r^m||_2 at exit */
    double rho_mean;       /* mean of ||r^(m+1)||/||r^(m)|| over m = 11..15 (0 if fewer cycles; if some of
                              those cycles were not checked, the per-cycle rate between the nearest
                              checked cycles around them) */
    double solve_ms;       /* device time of the solve (HIP events on the stream) */
} bcmg_solve_stats;

/* Thread-local message of the last failed call ("" if none). */
const char *bcmg_last_error(void);

/* Library version (major*100 + minor). */
int32_t bcmg_version(void);

/*
 * Device memory (not an operation of the paper: the plumbing that lets a
 * host framework own HBM).  Every device allocation the library makes
 * (problem hierarchies, batch tables, setup temporaries) goes through
 *   alloc(bytes, stream, ctx) -> pointer, 256-byte aligned, or NULL on failure
 *   free(ptr, bytes, stream, ctx)
 * stream is the hipStream_t on which the memory is used: frees are
 * stream-ordered (the memory may be handed out again only in that stream's
 * order, as with hipFreeAsync), and alloc must return memory usable in that
 * stream's order.  Both NULL (the default): a private stream-ordered pool per
 * device that keeps freed memory for reuse; the process's default pool is
 * not touched.  The source in effect when a problem is set up or a batch is
 * created serves it until it is destroyed, so changing it later does not
 * affect existing handles.  A NULL alloc result makes the calling setup or
 * batch call fail with BCMG_ERR_OOM.  Giving one callback without the other
 * is BCMG_ERR_INVALID.  The callbacks may be called from any thread that
 * calls the library, and must be safe for that.
 */
typedef void *(*bcmg_alloc_fn)(size_t bytes, void *stream, void *ctx);
typedef void (*bcmg_free_fn)(void *ptr, size_t bytes, void *stream, void *ctx);
bcmg_status bcmg_set_allocator(bcmg_alloc_fn alloc, bcmg_free_fn free, void *ctx);

/* Fill *opt with the defaults: V(2,1), coarsest N = 4, 100 cycles, FP64,
 * exponential-form dtau (Remark exptheta2D), K = 4, renormalised FW,
 * 128-node row segments. */
bcmg_status bcmg_default_options(bcmg_options *opt);

/*
 * Build the grid hierarchy for the level set phi sampled at the finest nodes.
 *   dim: 1, 2 or 3.  N: intervals per axis, a power of two with N >= 8
 *   and N <= 4096 (1D/2D) or 1024 (3D).
 *   phi_dev: (N+1)^dim FP64 node values, x fastest; read during the call only.
 *     Coarse levels take phi by injection (every coarse node is a fine node) and
 *     are classified on their own (Sec. 3.3: a node may be inactive on one
 *     level and a ghost on the next).
 *   stream: hipStream_t for every later call on this problem (NULL = default).
 * Per level the setup classifies nodes, compacts the ghost list in ascending
 * node order, computes each ghost's upwind stencil, projection Q = G - eta h n,
 * theta~ = eta and dtau (eqs. BCh, rel, DtauOptTheta), the extension band and
 * the coarsest-level inverse.  Returns BCMG_ERR_INVALID for bad sizes/options,
 * non-finite phi, or a phi that is negative at no node (a domain with no
 * unknowns).  Coarse levels with no INSIDE node are allowed: their correction
 * is zero.
 */
bcmg_status bcmg_setup(int32_t dim, int32_t N, const double *phi_dev, const bcmg_options *opt, void *stream,
                       bcmg_problem **out);

/* Release every device buffer of the problem (stream-ordered). */
bcmg_status bcmg_destroy(bcmg_problem *prob);

/* Number of grid levels (finest = 0). */
bcmg_status bcmg_num_levels(const bcmg_problem *prob, int32_t *levels);

/* Sizes of a level: intervals N, INSIDE and GHOST counts, extension band and
 * row-segment counts.  Any output pointer may be NULL. */
bcmg_status bcmg_level_info(const bcmg_problem *prob, int32_t level, int32_t *N, int64_t *n_inside,
                            int64_t *n_ghost, int64_t *n_band, int64_t *n_segments);

/* Copy the class array of a level ((N_l+1)^dim uint8, BCMG_* codes) to cls_dev. */
bcmg_status bcmg_classes(const bcmg_problem *prob, int32_t level, uint8_t *cls_dev);

/*
 * Ghost data of a level in ghost-list order (ascending node index); any
 * pointer may be NULL.
 *   idx_dev   int32[n_ghost]     node index
 *   code_dev  int32[n_ghost]     stencil code: bits 0-1,2-3,4-5 widths w_x,w_y,w_z
 *                                (1..3); bits 6,7,8 set when s_x,s_y,s_z = -1
 *                                (the stencil extends towards -s_k, upwind)
 *   eta_dev   double[n_ghost]    theta~ = |G-Q|/h (eq. DtauOptTheta)
 *   normal_dev double[3*n_ghost] unit normal n (from central differences of phi)
 *   q_dev     double[3*n_ghost]  projection Q = G - eta h n
 *   tau_dev   double[3*n_ghost]  local coordinates of Q along each stencil axis
 *   dtau_dev  double[n_ghost]    fictitious time step of the ghost row
 *   fallback_dev int32[n_ghost]  bit 0: the root search fell back to the first-order
 *                                distance; bit 1: a Neumann row with no admissible
 *                                block, replaced by (u_G - u_J)/h towards the first
 *                                INSIDE axis neighbour J
 * Neumann rows are the normal derivative of the tensor-product interpolant
 * at Q, sum_k n_k d/dx_k; their blocks may contain BOXDIR nodes.
 */
bcmg_status bcmg_ghost_info(const bcmg_problem *prob, int32_t level, int32_t *idx_dev, int32_t *code_dev,
                            double *eta_dev, double *normal_dev, double *q_dev, double *tau_dev, double *dtau_dev,
                            int32_t *fallback_dev);

/*
 * Stencil statistics of a level's ghost rows (Sec. 3.3, the widths of R8 and
 * the fallbacks above), counted on the host from the level's codes and
 * flags.  counts_host (27 int64, may be NULL): counts_host[k] is the number of
 * rows whose widths, sorted in decreasing order with missing axes taken as 1,
 * are (a, b, c) with k = 9 (3 - a) + 3 (3 - b) + (3 - c): k = 0 is (3,3,3),
 * 13 is (2,2,2), 26 is (1,1,1).  root_fallback_host / row_fallback_host (may
 * be NULL): rows with fallback bit 0 / bit 1 set.
 */
bcmg_status bcmg_ghost_stats(const bcmg_problem *prob, int32_t level, int64_t *counts_host,
                             int64_t *root_fallback_host, int64_t *row_fallback_host);

/*
 * Right-hand side of the finest level: f_dev (nodes; used on INSIDE nodes) and
 * gq_dev (n_ghost values g(Q) in ghost-list order, the boundary data at the
 * projections returned by bcmg_ghost_info; for Neumann rows the normal
 * derivative along each ghost's normal).  Both copied; NULL f means 0.
 */
bcmg_status bcmg_set_data(bcmg_problem *prob, const double *f_dev, const double *gq_dev);

/* u_dev[BOXDIR nodes] = gbox_dev (nodes; NULL means 0).  Other entries untouched. */
bcmg_status bcmg_fill_boundary(bcmg_problem *prob, const double *gbox_dev, double *u_dev);

/* One (nu1,nu2) cycle of the problem's shape (V or W) on u_dev (finest
 * level, FP64, in place).  INSIDE and GHOST entries are the unknowns, BOXDIR
 * entries must hold g_B, other entries are never read or written.  Sec. 2.1
 * (TGCS and its recursion with gamma = 1 or 2). */
bcmg_status bcmg_vcycle(bcmg_problem *prob, double *u_dev);

/* ||f - A u||_2 over INSIDE and GHOST rows of the finest level (host result). */
bcmg_status bcmg_residual_norm(bcmg_problem *prob, const double *u_dev, double *norm_host);

/*
 * bcmg_residual_norm for callers that cannot allocate device memory (code
 * under stream capture, tight serving loops, hosts that forbid allocation):
 * the same kernels and summation order, so the same result, but the norm's
 * partial sums, range record and result live in a static device array of the
 * library (4 MiB plus 32 bytes per device, held until the process ends); the
 * call allocates nothing.  It writes the residual into the problem's own
 * finest-level scratch, as bcmg_residual_norm does, and synchronises the
 * problem's stream.  Limit: at most 524287 row segments plus ghost chunks on
 * the finest level (bcmg_level_info; a 513^3 flower has about 8e4), else
 * BCMG_ERR_INVALID.  Every call on one device shares that device's array:
 * calls that overlap on one device (other threads or streams) race and must
 * be serialised by the caller.  BCMG_ERR_STATE if the device current at the
 * call is not the one the problem was set up on.
 */
bcmg_status bcmg_residual_norm_noalloc(bcmg_problem *prob, const double *u_dev, double *norm_host);

/*
 * Solve in place from the given u_dev until ||r^m|| <= rel_tol ||r^0||
 * (residual normalised by the first iteration, Sec. 3.3 comparison with AGMG).
 * In BCMG_MIXED mode each cycle is an FP64 residual, an FP32 V-cycle on the
 * correction with an FP64 coarse solve, and an FP64 update (iterative
 * refinement).  hist_host (max_cycles+1 doubles, may be NULL) receives
 * ||r^m|| for m = 0..cycles.  Returns the solve status.  The problem keeps
 * its work lists and captured cycles between calls, also when u_dev is
 * another array than the last call's.
 *
 * Convergence checks.  A check is the residual norm over the finest level
 * (in BCMG_MIXED mode also the update and the FP32 right-hand side of the
 * next correction cycle).  With check_interval k > 1 the solve runs blocks
 * of up to k cycles per check (in BCMG_MIXED mode: the block's FP32 cycles
 * iterate on one correction equation) while the rate observed between the
 * last two host-read checks predicts at least two more cycles after the
 * block; the first two cycles and the last two predicted are checked one by
 * one.  A
 * cycle not followed by a check
 * leaves NaN in hist_host.  Unchecked cycles count in cycles and max_cycles.
 * The solve can run past the cycle where a per-cycle check would have
 * stopped (by at most k - 1 cycles) only when the rate improves by more than
 * the prediction allows.
 */
bcmg_status bcmg_solve(bcmg_problem *prob, double *u_dev, double rel_tol, bcmg_solve_stats *stats_host,
                       double *hist_host);

/* ---- single steps of the cycle on caller buffers (FP64), level l ---------- */

/* steps x (red-black Gauss-Seidel on INSIDE nodes, then one Jacobi ghost
 * relaxation u_G += dtau_G (rhs_G - sum w u), eqs. GSLEX_2D in red-black
 * order, rel, 2Ddiri:P); rhs holds f on INSIDE and the ghost-row data on GHOST. */
bcmg_status bcmg_level_smooth(bcmg_problem *prob, int32_t level, double *u_dev, const double *rhs_dev,
                              int32_t steps);

/* r = rhs - A u on INSIDE and GHOST rows (r elsewhere untouched); optional norm. */
bcmg_status bcmg_level_residual(bcmg_problem *prob, int32_t level, const double *u_dev, const double *rhs_dev,
                                double *r_dev, double *norm_host);

/* Normal extension of the GHOST values of v into the OUTSIDE nodes within
 * Chebyshev distance K of a ghost (K upwind Jacobi sweeps from 0, Sec. 3.3
 * transfer operators); other OUTSIDE entries of v must already be 0. */
bcmg_status bcmg_level_extend(bcmg_problem *prob, int32_t level, double *v_dev);

/* rhs_coarse (level+1) from the extended residual r_fine (level), eq.
 * coarseFW and Sec. 3.3: renormalised FW kept separate for interior and ghost
 * rows.  Written on coarse INSIDE and GHOST nodes only. */
bcmg_status bcmg_level_restrict(bcmg_problem *prob, int32_t level, const double *rfine_dev, double *rhs_coarse_dev);

/* u_fine += P e_coarse on fine INSIDE and GHOST nodes (multilinear); e_coarse
 * (level+1) must hold 0 on BOXDIR and OUTSIDE nodes; its OUTSIDE band entries
 * are overwritten by the extension first (Sec. 3.3). */
bcmg_status bcmg_level_prolong(bcmg_problem *prob, int32_t level, double *ecoarse_dev, double *ufine_dev);

/* Exact solve on the coarsest level (dense inverse built at setup; BOXDIR
 * values of the coarsest level are 0). */
bcmg_status bcmg_coarse_solve(bcmg_problem *prob, double *u_dev, const double *rhs_dev);

/* ---- batches: many independent problems advanced together ---------------- */

/*
 * A batch advances every active slot by whole V-cycles with one set of
 * launches per cycle (levels aligned at the coarsest grid), captured once in a
 * hipGraph and replayed.  All problems of a batch share dim and precision.
 * Problems stay owned by the caller; u_dev of each slot is kept until removal.
 */
bcmg_status bcmg_batch_create(int32_t capacity, void *stream, bcmg_batch **out);
bcmg_status bcmg_batch_destroy(bcmg_batch *b);

/* Add a problem (after bcmg_set_data) with its solution buffer and tolerance;
 * computes ||r^0|| and returns the slot. */
bcmg_status bcmg_batch_add(bcmg_batch *b, bcmg_problem *prob, double *u_dev, double rel_tol, int32_t *slot);

/* Restart every occupied slot from the current contents of its u_dev
 * (recomputes ||r^0||); work lists and graphs are kept. */
bcmg_status bcmg_batch_restart(bcmg_batch *b);

/* Drop a slot (its problem and u_dev are released to the caller). */
bcmg_status bcmg_batch_remove(bcmg_batch *b, int32_t slot);

/* Advance every active slot by `cycles` V-cycles (converged slots are left
 * untouched), then copy each slot's state to the host: active_host[capacity]
 * = 1 while a slot still iterates, 0 when done or free.  Synchronises. */
bcmg_status bcmg_batch_step(bcmg_batch *b, int32_t cycles, int32_t *active_host);

/* Step until no slot is active or max_steps steps were taken. */
bcmg_status bcmg_batch_run(bcmg_batch *b, int32_t cycles_per_step, int32_t max_steps);

/* Final state of a slot (valid once inactive). hist_host may be NULL. */
bcmg_status bcmg_batch_stats(bcmg_batch *b, int32_t slot, bcmg_solve_stats *stats_host, double *hist_host);

/* Device bytes a problem of this size would need (for admission control): an
 * upper bound of what bcmg_problem_bytes reports after bcmg_setup, for
 * Dirichlet and Neumann rows alike (its model: the node arrays of every level,
 * a surface term for ghost and band records, and the arena's chunking). */
bcmg_status bcmg_estimate_bytes(int32_t dim, int32_t N, int32_t precision, int64_t *bytes);

/* Batch tuning parameters (take effect at the next step). */
#define BCMG_PARAM_COARSE_NODES 1 /* levels with at most this many nodes run in one workgroup per problem (default 5000;
                                     lowered as needed so that they fit the LDS budget) */
#define BCMG_PARAM_LDS_BYTES 2    /* LDS bytes that workgroup may hold its levels in (default and maximum 153600;
                                     0 keeps them in HBM) */
#define BCMG_PARAM_SWEEP_PAIR_SEGS 3 /* FP32 red-black launches over split-layout levels (BCMG_LAYOUT_SPLIT) with
                                        at least this many row segments give each wavefront four segments and
                                        each lane four nodes of a colour (default 1: all of them; a larger value
                                        keeps smaller levels on one segment per wavefront); the same bits */

bcmg_status bcmg_batch_set_param(bcmg_batch *b, int32_t param, int64_t value);

/* Bytes of device memory held by a problem. */
bcmg_status bcmg_problem_bytes(const bcmg_problem *prob, int64_t *bytes);

/* ---- instrumentation ------------------------------------------------------ */

/* While enabled (process-wide), batch and solve calls launch their cycles
 * directly instead of replaying a graph, with a HIP event pair around every
 * launch of the finest-level red-black sweep on the solver's stream;
 * bcmg_timing_read returns the number of timed launches, their summed
 * duration in ms and the INSIDE nodes of the finest level swept per launch.
 * Enabling or disabling resets the counters. */
bcmg_status bcmg_timing_enable(int32_t on);
bcmg_status bcmg_timing_read(int64_t *launches, double *total_ms, int64_t *inside_nodes_per_launch);

/* Back-to-back finest-level red-black sweeps (reps red + black pairs),
 * launched directly between one HIP event pair on the problem's stream:
 * *ms_host is the elapsed time, so the time per colour launch is
 * *ms_host / (2 reps).  FP64 problems sweep a scratch copy of u_dev (u_dev
 * is not modified); mixed-precision problems sweep the FP32 arrays of their
 * correction cycle (u_dev may be NULL; a later solve starts them afresh). */
bcmg_status bcmg_timing_sweeps(bcmg_problem *prob, const double *u_dev, int32_t reps, double *ms_host);

#ifdef __cplusplus
}
#endif

#endif /* BCMG_H */
