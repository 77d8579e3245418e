/*
 * rw.h -- C ABI of the refined-wall Stokes solver for AMD MI355X (gfx950).
 *
 * Method: Zhang, Gillman & Veerapaneni, "A fast direct solver for integral
 * equations on locally refined boundary discretizations and its application
 * to multiphase flow simulations" (arXiv:2108.07205).
 *
 * The library solves the interior Stokes Dirichlet problem (Sec. 2.1, eq.
 * model_bvp) on a closed star curve with the double-layer representation,
 * Nystrom-discretized as A = -1/2 I + D + N (eqs. interior_BIE_discretized2
 * and null), on a wall whose discretization is locally refined (Sec. 3.1).
 * Per refinement it follows Algorithm 1 (Sec. 3.2):
 *   precompute: Q ~= L R (Secs. 3.3-3.4), A_pp^{-1}, X = A~^{-1} L and the
 *               Woodbury operator W = I + R X with its LU;
 *   solve:      y = A~^{-1} g_ext (reference HBS inverse + A_pp^{-1}) and
 *               tau_ext = y - X W^{-1} R y (eq. wood),
 * followed by FP64 iterative refinement on the exact refined Nystrom residual.
 *
 * Conventions (all calls):
 *  - Return value: RW_OK (0) or a negative RW_E* code; rw_last_error() gives
 *    a message.  A call that fails leaves no partially built handle behind.
 *  - Handles (rw_ctx, rw_wall, rw_refined) are opaque and library-owned;
 *    free them with the matching free or destroy call.  A wall must outlive
 *    the refined handles made from it; a ctx must outlive its walls.
 *  - Arrays named *_dev are device pointers (HBM of the ctx's device),
 *    owned by the caller, read/written on the ctx's HIP stream.  Arrays named
 *    *_host are host pointers owned by the caller.
 *  - Unknowns are node-major with (u_x, u_y) interleaved: unknown 2i is the
 *    x component at node i, 2i+1 the y component.  Nodes follow the panel
 *    order of the discretization (increasing curve parameter theta), 16 (or
 *    `order`) Gauss-Legendre nodes per panel.
 *  - Multi-column arrays are column-major with leading dimension 2*N (no
 *    padding).
 *  - Calls on one ctx are not thread-safe; use one ctx per host thread.
 */
#ifndef RW_H
#define RW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rw_ctx rw_ctx;
typedef struct rw_wall rw_wall;
typedef struct rw_refined rw_refined;

enum rw_status {
  RW_OK = 0,
  RW_EINVAL = -1,     /* bad argument: ids out of range, duplicates, level < 0 or > 8, nrhs <= 0, ... */
  RW_ENOMEM = -2,     /* the request does not fit the ctx's HBM budget, or hipMalloc failed */
  RW_ESINGULAR = -3,  /* zero / non-finite pivot in W, A_pp or an HBS node block */
  RW_ENOCONV = -4,    /* iterative refinement did not reach the requested residual */
  RW_EDEVICE = -5     /* a HIP runtime call or a kernel reported an error */
};

/* Storage precision of the reference HBS generators read by the solve's
 * applies of A_oo^{-1} (the FP64 copy is always kept and used for X = A~^{-1}
 * L; the residual, W and its inverse, and the root block stay FP64).  FP32
 * and BF16 applies accumulate in FP64 with one right-hand side and in FP32
 * on the matrix cores with many; FP64 iterative refinement (or GMRES)
 * recovers the digits. */
enum rw_precision { RW_F64 = 0, RW_F32 = 1, RW_BF16 = 2 };

/* Solver of rw_solve after the refinement's factors are built. */
enum rw_solver {
  RW_SOLVE_IR = 0,    /* Richardson refinement: tau += M^{-1} (g - A_nn tau), M^{-1} the Woodbury solve */
  RW_SOLVE_GMRES = 1  /* GMRES on the exact A_nn, right-preconditioned by the Woodbury solve (Sec. 4) */
};

/* How the products A_nn tau of the residual (and of GMRES) are formed.  Both
 * are the Nystrom operator of Sec. 2 in FP64 with no approximation beyond
 * rounding: the expansions cut the multipole series of the double layer
 * (Sec. 4.2 names fast products of this kind) where the dropped terms are
 * below 1e-17 of the cluster's own contribution. */
enum rw_resid {
  RW_RESID_AUTO = 0,   /* RW_RESID_EXPAND from 4096 nodes, RW_RESID_PAIRS below */
  RW_RESID_PAIRS = 1,  /* every pair of nodes summed directly */
  RW_RESID_EXPAND = 2  /* clusters of 256 consecutive nodes farther than 3 cluster radii from a group of
                          128 targets through their multipole expansions (at most 40 terms), the others
                          pair by pair; from 32768 nodes, far clusters of 2048 nodes by one expansion each */
};

/* Star curve gamma(theta) = (1 + a cos(m theta)) (cos theta, sin theta),
 * theta in [0, 2 pi), counter-clockwise (a = 0: unit circle). */
typedef struct {
  double a;
  int32_t m;
} rw_curve;

/* Solver options of a ctx (defaults in brackets). */
typedef struct {
  double ir_tol;             /* stop refinement when ||g - A tau|| / ||g|| <= ir_tol, per column [1e-13] */
  int32_t ir_maxit;          /* max refinement corrections; 0 = plain Woodbury solve [6] */
  int32_t sketch_cols;       /* columns of the random sketch used for the row IDs of Q, 32..128 [64] */
  uint64_t seed;             /* seed of the sketching matrix (counter-based, reproducible) [0x5eed] */
  int32_t app_dense_max_nodes; /* A_pp^{-1} by dense LU up to this many added nodes, else by an HBS
                                  inverse built on the GPU (Algorithm 1 step 2) [1024] */
  int32_t far_field;         /* 1: split the kept nodes at a circle around the refined arc (Sec. 3.3)
                                and sketch the far part of Q through multipole / local expansions,
                                the near part exactly (used when at most half the kept nodes are
                                near); 0: sketch the whole blocks of Q exactly [1] */
  int32_t hbs_merge;         /* binary tree levels merged into one level of the reference HBS tree built
                                by the next rw_wall_build, 1..4 (1: binary tree; 2: four children per
                                node): fewer dependent level sweeps per apply [2] */
  int32_t solver;            /* RW_SOLVE_IR or RW_SOLVE_GMRES [RW_SOLVE_IR]; with GMRES, ir_maxit caps the
                                Krylov iterations over all restarts and ir_tol is the same residual test */
  int32_t gmres_restart;     /* GMRES: Krylov dimension before a restart, 1..256 [30] */
  int32_t gmres_precond;     /* GMRES: 1 = preconditioned by the Woodbury solve (Sec. 4, eq.
                                left_precond_general applied on the right), 0 = plain GMRES on A_nn [1] */
  int32_t mfma_from;         /* multi-RHS applies of a wall's inverse on the matrix cores from this many
                                right-hand sides; 0 = the crossover rw_wall_build measured [0] */
  int32_t test_singular;     /* test hook, 0 in normal use [0]: 1 = zero the first column of W = I + R X
                                before its inversion, whose pivot check then reports RW_ESINGULAR; 2 =
                                zero the first column of a dense A_pp before its LU, whose pivot check
                                then hands A_pp to the GPU-built HBS inverse */
  int32_t one_stream;        /* 1 = every step of rw_refine and rw_solve on the ctx's own stream, with no
                                helper thread and no side streams (the A_pp inverse then runs before the
                                compression of Q instead of beside it): for contexts that run side by side,
                                each on one hardware queue, such as the slots of rw_server_create [0] */
  int32_t resid_mode;        /* an rw_resid value [RW_RESID_AUTO] */
} rw_options;

/* Counts and timings reported by rw_refine / rw_solve. */
typedef struct {
  int64_t n_k, n_c, n_p;     /* kept / cut / added node counts (Sec. 3.1) */
  int32_t k_k, k_p, k;       /* ranks of the k-row and p-row IDs of Q, k = k_k + k_p */
  int32_t ir_iters;          /* refinement corrections applied by the last rw_solve */
  double resid;              /* max over columns of ||g - A_nn tau|| / ||g|| after the last rw_solve */
  double t_refine_ms;        /* host time of the last rw_refine / rw_coarsen (until it returned,
                                which is before its last device work ends) */
  double t_solve_ms;         /* wall time of the last rw_solve */
  int64_t n_near;            /* kept nodes sketched exactly by the far-field split, -1 if Q's blocks
                                were sketched exactly as a whole */
  int64_t app_entries;       /* generator entries of the GPU-built HBS inverse of A_pp (0 for the dense
                                LU or no added nodes); set once the refinement's device-side checks
                                have been read (by the first rw_solve / rw_residual on the handle) */
  int32_t app_max_rank;      /* largest node rank of that HBS inverse (0 as above) */
  double app_lu_mult;        /* largest |entry of L| of the unpivoted dense LU of A_pp (+inf for a zero
                                pivot, 0 when no dense LU ran); above 1e3 the dense LU is dropped and
                                A_pp^{-1} is the GPU-built HBS inverse (app_entries > 0) instead */
} rw_info;

/* Outcome of one rw_solve (Algorithm 1 solve steps + refinement). */
typedef struct {
  int32_t ir_iters;          /* refinement corrections applied (RW_SOLVE_IR) or Krylov iterations over all
                                restarts, summed over the columns (RW_SOLVE_GMRES) */
  int32_t k;                 /* rank k = k_k + k_p of the Woodbury update used */
  double resid;              /* max over columns of ||g - A_nn tau|| / ||g|| on return */
  double resid_direct;       /* the same for the plain Woodbury solution (before any correction; with
                                RW_SOLVE_GMRES after the first Krylov step) */
  double t_solve_ms;         /* wall time of the call */
} rw_solve_info;

/* Reference-wall statistics reported by rw_wall_stats. */
typedef struct {
  int64_t n_nodes;           /* N_o */
  int32_t n_levels;          /* tree levels below the root (root = level 0, leaves = level n_levels) */
  int32_t max_rank;          /* largest skeleton size of any tree node */
  int64_t gen_entries;       /* sum over nodes of |E| + |F| + |G| (the generators one apply reads) */
  int64_t gen_bytes_f64;     /* 8 * gen_entries */
  double t_build_ms;         /* host + device time of rw_wall_build */
  int32_t mfma_from_f64;     /* right-hand-side count from which multi-RHS applies of this wall's inverse
                                run on the FP64 matrix cores, measured by rw_wall_build (65 or more:
                                never below 64 in the measurement) */
  int32_t mfma_from_f32;     /* the same for FP32 generators (0 when the wall has none) */
} rw_wall_stats;

/* ---- context ---------------------------------------------------------- */

/* Create a ctx bound to HIP device `device` and stream `hip_stream`
 * (a hipStream_t; NULL = the legacy default stream).  `hbm_budget_bytes`
 * caps the device memory the library itself allocates for this ctx
 * (0 = no cap).  Errors: RW_EINVAL (bad device), RW_EDEVICE. */
int rw_ctx_create(rw_ctx** out, int device, void* hip_stream, size_t hbm_budget_bytes);
void rw_ctx_destroy(rw_ctx* ctx);
/* Message of the last error on this ctx ("" if none).  Valid until the next call. */
const char* rw_last_error(const rw_ctx* ctx);
/* Message of the last error of a failed rw_ctx_create (ctx does not exist yet). */
const char* rw_create_error(void);
int rw_set_options(rw_ctx* ctx, const rw_options* opt);
int rw_get_options(const rw_ctx* ctx, rw_options* opt);
/* Bytes the library currently holds on the device for this ctx, including
 * blocks kept for reuse by its caching allocator (freed handles return their
 * device memory to that cache, so a steady refine / solve loop stops calling
 * hipMalloc once warm). */
size_t rw_ctx_bytes(const rw_ctx* ctx);
/* Return the cached (unused) device blocks of this ctx to the HIP runtime. */
int rw_ctx_trim(rw_ctx* ctx);

/* Phase profiler: when enabled, every step of Algorithm 1 (a1_geometry,
 * a2_sketch, a2_row_id, a2_interp_rows, a3_app_assemble, a3_app_lu, a4_X,
 * a5_W, a6_hbs_apply, a6_app_solve, a7_woodbury, a8_residual) is bracketed by
 * HIP events on the ctx stream; rw_profile_json writes
 *   {"phase": {"ms": total, "calls": n, "flops": algorithmic flops,
 *              "bytes": algorithmic HBM bytes}, ...}
 * into buf (NUL-terminated, truncated to len) and returns the length needed
 * including the NUL (or a negative error). */
int rw_profile_enable(rw_ctx* ctx, int on);
int rw_profile_reset(rw_ctx* ctx);
int64_t rw_profile_json(rw_ctx* ctx, char* buf, int64_t len);

/* ---- reference wall (static; Sec. 3.2: Algorithm 1 takes a fast direct
 *      solver of the reference discretization as its input) ------------- */

/* Discretize the curve with n_panels Gauss-Legendre panels of `order`
 * nodes, uniform in theta, and build the HBS compressed inverse A_oo^{-1}
 * (tree of contiguous arcs, leaves of `leaf_nodes` nodes; interpolative
 * decompositions at relative tolerance id_tol, Definition 3.1).  The
 * generators are uploaded to HBM.  The tree has the fewest binary levels
 * whose leaves hold at most leaf_nodes nodes (2^L leaves of consecutive
 * nodes, their sizes differing by at most one).  Requirements: order in
 * [2, 32], n_panels >= 2, leaf_nodes a positive multiple of order.
 * Errors: RW_EINVAL, RW_ENOMEM, RW_ESINGULAR, RW_EDEVICE. */
int rw_wall_build(rw_ctx* ctx, const rw_curve* curve, int32_t n_panels, int32_t order,
                  int32_t leaf_nodes, double id_tol, int32_t precision, rw_wall** out);
void rw_wall_free(rw_wall* wall);
int rw_wall_stats_get(const rw_wall* wall, rw_wall_stats* st);
/* Node arrays of the reference discretization (host, caller-owned, length
 * 2*N_o for xy/normals, N_o for weights; NULL arrays are skipped).
 * *n_nodes in: capacity in nodes, out: N_o. */
int rw_wall_nodes(const rw_wall* wall, double* xy_host, double* normals_host,
                  double* weights_host, int64_t* n_nodes);

/* x = A_oo^{-1} b with the HBS inverse (Algorithm 1, solve step 1, first
 * block).  b_dev, x_dev: 2*N_o x nrhs column-major, may not alias.
 * Errors: RW_EINVAL (nrhs <= 0), RW_ENOMEM, RW_EDEVICE. */
int rw_hbs_apply(rw_wall* wall, const double* b_dev, int32_t nrhs, double* x_dev);

/* One-RHS x = A_oo^{-1} b, as rw_hbs_apply with nrhs = 1, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): no hipMalloc, hipFree or
 * other allocating call.  Its partial vectors live in a file-scope device
 * array of 2^21 doubles (16 MiB) that each device holds until the process
 * ends; walls whose apply needs more are rejected with RW_EINVAL.  Every
 * call on a device shares that array (each call writes every partial before
 * reading it, so nothing needs clearing), so calls that overlap on one GPU
 * (several ctxs or streams) race: order them.  b_dev, x_dev: 2*N_o doubles
 * (one column), may not alias; enqueued on the ctx stream, not synchronized,
 * no profiler events.  Errors: RW_EINVAL (null arrays, wall too large),
 * RW_EDEVICE. */
int rw_hbs_apply_noalloc(rw_wall* wall, const double* b_dev, double* x_dev);

/* ---- refinement (per time step; Algorithm 1 pre-computation) ------------ */

/* Refine reference panels panel_ids[i] into 2^levels[i] equal-theta
 * children (levels[i] = 0 keeps the panel but still routes it through the
 * extended system), then build Q ~= L R, A_pp^{-1}, X = A~^{-1} L and the LU
 * of W = I + R X.  n_sel = 0 gives the unrefined wall (k = 0).
 * q_tol: relative tolerance of the row IDs of Q's k-rows and p-rows
 * (Definition 3.1; Secs. 3.3-3.4), in (0, 1); q_tol <= 0 takes the wall's
 * id_tol.  The HBS inverse of A_pp (large refinements) uses the wall's id_tol.
 * Errors: RW_EINVAL (ids out of [0, n_panels), duplicates, levels outside
 * [0, 8]), RW_ENOMEM, RW_ESINGULAR, RW_EDEVICE.
 * Asynchrony: the call returns once the last part of the pre-computation
 * (the A_pp^{-1} build's top levels, X and W) is enqueued, on a second
 * stream of the ctx that the later calls on the handle wait for; work the
 * caller enqueues on the ctx's stream meanwhile (Stokeslet data, the solve)
 * can start beside it.  The checks
 * that read device results (a zero pivot in W or in an HBS node block, an
 * HBS rank reaching the sketch size) are then made by the first of
 * rw_solve, rw_solve_batch or rw_residual on the handle, or by the next
 * rw_refine / rw_coarsen on the ctx; a failure found there is returned by
 * that handle's rw_solve / rw_solve_batch / rw_residual (RW_ESINGULAR) from
 * then on.  With the ctx profiler on, rw_refine waits and reports it
 * itself.  rw_refined_free waits for the handle's device work. */
int rw_refine(rw_wall* wall, const int32_t* panel_ids_host, const int32_t* levels_host,
              int32_t n_sel, double q_tol, rw_refined** out);
/* rw_refine on another ctx of the wall's device: the refinement's device
 * work, memory and later calls (rw_solve, rw_residual, rw_stokeslet_rhs,
 * rw_refined_free) use ctx's stream and allocator and ctx's own workspace for
 * applies of the wall's reference inverse, which is only read.  Several
 * host threads, each with its own ctx, can thus refine and solve against
 * one resident wall at once (the wall's own ctx must not be used meanwhile
 * for rw_hbs_apply or rw_solve_batch, whose workspace is the wall's).  The
 * wall must outlive the handle; ctx must outlive the handle.  Errors as
 * rw_refine, and RW_EINVAL when ctx is on another device. */
int rw_refine_on(rw_ctx* ctx, rw_wall* wall, const int32_t* panel_ids_host, const int32_t* levels_host,
                 int32_t n_sel, double q_tol, rw_refined** out);
/* Coarsen: give panel_ids_host[i] back its reference discretization and
 * redo the pre-computation (with the handle's q_tol) for the remaining refinement (coarsening all
 * refined panels returns the reference problem).  Ids that are not refined
 * are an error (RW_EINVAL).  On error the handle is unchanged. */
int rw_coarsen(rw_refined* ref, const int32_t* panel_ids_host, int32_t n_sel);
void rw_refined_free(rw_refined* ref);
int rw_refined_info(const rw_refined* ref, rw_info* info);
/* Node arrays of the refined discretization I_n (host), as rw_wall_nodes. */
int rw_nodes(const rw_refined* ref, double* xy_host, double* normals_host,
             double* weights_host, int64_t* n_nodes);

/* ---- solve (Algorithm 1 solve steps + FP64 refinement) ------------------ */

/* tau = A_nn^{-1} g for nrhs right-hand sides: Woodbury solve (eq. wood)
 * then iterative refinement with the exact refined Nystrom residual until
 * ||g - A_nn tau|| / ||g|| <= ir_tol (per column) or ir_maxit corrections.
 * With ir_maxit >= 1 the first correction is always taken (it is enqueued
 * before the first residual is read back).  With solver = RW_SOLVE_GMRES:
 * restarted GMRES per column from tau = 0 on the exact A_nn (its products by
 * the residual kernel), right-preconditioned by the Woodbury solve unless
 * gmres_precond = 0, modified Gram-Schmidt applied twice per step, until the
 * same residual test or ir_maxit iterations; the residual is recomputed at
 * each restart and at the end.
 * g_dev, tau_dev: 2*N_n x nrhs column-major, may not alias.  info_host: NULL
 * or a caller-owned rw_solve_info that receives the outcome (also on
 * RW_ENOCONV).  The stream is synchronized before return.  Errors:
 * RW_EINVAL, RW_ENOMEM, RW_ENOCONV (result written, residual above
 * tolerance), RW_ESINGULAR (the refinement's deferred checks failed; tau is
 * not a solution), RW_EDEVICE. */
int rw_solve(rw_refined* ref, const double* g_dev, int32_t nrhs, double* tau_dev,
             rw_solve_info* info_host);

/* Several refinements of one wall in one call (Algorithm 1 solve steps for
 * each; Sec. 3.2: every refinement reuses the same reference inverse).  The
 * A_oo^{-1} applies of all instances are stacked into one multi-RHS apply per
 * sweep, so the reference generators are streamed once for the whole batch;
 * each instance then takes refinement corrections until its own columns
 * meet ir_tol (or ir_maxit).  inst: n_inst distinct handles refined from the
 * same wall (library-owned); g_dev[i], tau_dev[i]: 2*N_n(i) x nrhs[i]
 * column-major device arrays (caller-owned, g and tau may not alias);
 * info_host: NULL or n_inst entries that receive each instance's rw_info.
 * The stream is synchronized before return.  Errors: RW_EINVAL (null or
 * repeated handles, handles of different walls, nrhs <= 0), RW_ENOMEM,
 * RW_ENOCONV (all results written; at least one instance stopped above the
 * tolerance), RW_ESINGULAR (an instance's deferred refinement checks
 * failed), RW_EDEVICE.  The instances must have been refined on the wall's
 * own ctx (rw_refine), whose stream runs the batch. */
int rw_solve_batch(rw_refined* const* inst, int32_t n_inst, const double* const* g_dev,
                   const int32_t* nrhs, double* const* tau_dev, rw_info* info_host);

/* r = g - A_nn tau on the refined discretization (the Nystrom operator of
 * Sec. 2 in FP64, entries generated on the fly; far node clusters through
 * their multipole expansions as rw_options.resid_mode selects).  Shapes as
 * rw_solve.  Enqueued on the ctx's stream (not synchronized).  Errors:
 * RW_EINVAL, RW_ENOMEM, RW_ESINGULAR (the refinement's deferred checks
 * failed), RW_EDEVICE. */
int rw_residual(rw_refined* ref, const double* g_dev, const double* tau_dev,
                int32_t nrhs, double* r_dev);

/* Boundary data of exterior Stokeslets (eq. stokeslet, mu = 1) at the refined
 * nodes: g(x_i) = sum_m S(x_i, z_m) f_m.  z_host, f_host: n_src x 2 row-major
 * (host; copied before return).  g_dev: 2*N_n (one column), written on the
 * ctx's stream (not synchronized).  Errors: RW_EINVAL, RW_EDEVICE. */
int rw_stokeslet_rhs(rw_refined* ref, const double* z_host, const double* f_host,
                     int32_t n_src, double* g_dev);

/* ---- refinement reuse across time steps (Sec. 5.3: several snapshots can
 *      use the same refinement) --------------------------------------- */

typedef struct rw_refcache rw_refcache;

/* A cache of refinements of `wall` (n_panels reference panels; the wall's
 * ctx runs them), at most `capacity` of them.  rw_refcache_get serves a
 * request with a cached refinement that covers it (every requested panel
 * refined at least as deep; the least refined such one); a miss refines
 * the requested panels widened by `margin` panels on both sides (each at
 * the deepest requested level within margin panels; runs whose widened
 * ranges touch form one region), caches it and frees the least recently
 * used one when full.  q_tol as rw_refine.  Errors: RW_EINVAL. */
int rw_refcache_create(rw_wall* wall, int32_t n_panels, int32_t capacity, int32_t margin, double q_tol,
                       rw_refcache** out);
/* *out: a refined handle owned by the cache (do not free it), valid until
 * the next rw_refcache_get on the cache or rw_refcache_destroy.  Its
 * discretization is the covering one: sample right-hand sides on its nodes
 * (rw_nodes, rw_stokeslet_rhs); rw_refcache_panels lists its refined
 * panels.  *hit (may be NULL): 1 if a cached refinement served it.  Errors
 * as rw_refine. */
int rw_refcache_get(rw_refcache* c, const int32_t* panel_ids_host, const int32_t* levels_host, int32_t n_sel,
                    rw_refined** out, int32_t* hit);
/* Refined panels and levels of a handle of the cache; *n in: capacity
 * (NULL arrays: size query), out: count.  Errors: RW_EINVAL. */
int rw_refcache_panels(const rw_refcache* c, const rw_refined* ref, int32_t* ids_host, int32_t* levels_host,
                       int32_t* n);
void rw_refcache_stats(const rw_refcache* c, int64_t* hits, int64_t* misses, int32_t* held);
void rw_refcache_destroy(rw_refcache* c);
const char* rw_refcache_error(const rw_refcache* c);

/* ---- serving (the time-stepping workflow of Sec. 5.3 served to many
 *      independent requests against one resident wall) ----------------- */

typedef struct rw_server rw_server;

/* Outcome of one served request. */
typedef struct {
  int32_t status;            /* RW_OK or the request's error code (RW_ENOCONV: result written) */
  int32_t slot;              /* slot that ran it */
  int32_t ir_iters;          /* refinement corrections (or GMRES iterations) */
  int32_t k;                 /* Woodbury rank */
  int64_t n_nodes;           /* refined nodes N_n */
  double resid;              /* max over columns of ||g - A_nn tau|| / ||g|| */
  double t_queue_ms;         /* submission to start */
  double t_run_ms;           /* start to end (refine, data, solve, copy back) */
} rw_request_info;

/* A server of `slots` worker threads (1..16), each with a ctx and stream of
 * its own (the options of `ctx` copied; with more than one slot, each slot's
 * ctx keeps to its one stream: one_stream = 1), that run whole requests against
 * `wall` (n_panels reference panels; built on ctx, resident, only read):
 * rw_refine_on, Stokeslet data, rw_solve, result copied back.  Requests
 * leave the queue in order as soon as a slot is free and the device memory
 * they are estimated to need fits hbm_budget_bytes (0: no cap) beside the
 * requests in flight, so the device work of up to `slots` requests of any
 * size overlaps.  ctx and wall must outlive the server.  Errors: RW_EINVAL,
 * RW_EDEVICE, or a slot ctx's creation error; rw_server_error(NULL) has the
 * message. */
int rw_server_create(rw_ctx* ctx, rw_wall* wall, int32_t n_panels, int32_t slots, size_t hbm_budget_bytes,
                     rw_server** out);
/* Queue a request: refine panel_ids_host[i] by levels_host[i] and solve for
 * nrhs right-hand sides, column r the velocity of the n_src Stokeslets
 * z_host / f_host rows r*n_src .. r*n_src + n_src - 1 (x, y pairs; copied
 * before return).  *id: the request's ticket for rw_server_wait.  Errors:
 * RW_EINVAL, RW_ENOMEM (the request could never fit the budget). */
int rw_server_submit(rw_server* sv, const int32_t* panel_ids_host, const int32_t* levels_host, int32_t n_sel,
                     const double* z_host, const double* f_host, int32_t n_src, int32_t nrhs, int64_t* id);
/* Block until request `id` is done; copy its tau (2 N_n x nrhs column-major,
 * refined node order) to tau_host (NULL: discard; cap: doubles available)
 * and its outcome to info (NULL: skip).  Returns the request's status, or
 * RW_EINVAL for an unknown ticket or a too small tau_host. */
int rw_server_wait(rw_server* sv, int64_t id, double* tau_host, int64_t cap, rw_request_info* info);
/* Waits for the requests still queued or running, then frees the slots. */
void rw_server_destroy(rw_server* sv);
/* Last error message of sv (NULL: of the last failed rw_server_create). */
const char* rw_server_error(const rw_server* sv);

#ifdef __cplusplus
}
#endif
#endif /* RW_H */
