/*
 * rs.h - C ABI of the MI355X (gfx950) recursive-skeletonization solver for the
 * 2D Stokes double-layer boundary integral equation on multiply-connected
 * domains (Ryan & Damle, "Parallel skeletonization for integral equations in
 * evolving multiply-connected domains").
 *
 * The operator (Section 3.1, eq. backwardeq) is the augmented system
 *
 *     [ lambda I + D + N   H ] [ mu     ]   [ f ]
 *     [ Psi^T             -I ] [ alpha  ] = [ 0 ]
 *                              [ beta   ]
 *
 * with D the stresslet double layer (eq. stokesbie), N the rank-one
 * completion (eq. null-spaceop), H the Stokeslet/rotlet columns of each hole
 * (eq. completed) and Psi the rigid motions of each hole (eq. null-space).
 * lambda I + D + N is factored by recursive skeletonization (Sections
 * 2.2-2.7) and the border is eliminated as in Section 3.2 (eq. partition).
 *
 * Conventions shared by every entry point:
 *  - Node arrays are host pointers in float64, row-major [n][2] for
 *    2-vectors.  Unknown 2j is the x-component of the density at node j and
 *    2j+1 its y-component; the 3p augmented unknowns follow, per hole h in
 *    the order (alpha_h1, alpha_h2, beta_h).
 *  - Normals are unit vectors pointing out of the fluid: outward on the
 *    outer curve, into each hole.  Curvature is signed: positive where the
 *    curve bends away from that normal.  curve_id is 0 on the outer curve
 *    and h (1..p) on hole h.
 *  - Inputs are copied during the call; the caller keeps ownership of every
 *    pointer it passes.  Outputs are caller-allocated.  The context owns all
 *    device memory it allocates and frees it in rs_destroy.
 *  - No exception crosses the ABI.  Every call returns an rs_status; on any
 *    status other than RS_OK, rs_last_error() describes the failure and the
 *    caller's output arrays are left untouched unless stated otherwise.
 *  - A context is not thread-safe and is bound to the HIP device that was
 *    current when it was built.
 */
#ifndef RS_MI355X_H
#define RS_MI355X_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rs_ctx rs_ctx;

typedef enum {
  RS_OK = 0,
  RS_ERR_ARG = 1,          /* invalid argument (non-finite value, bad size, bad id, NULL) */
  RS_ERR_STATE = 2,        /* call out of order (e.g. solve before factor)               */
  RS_ERR_ALLOC = 3,        /* device or host allocation failed                           */
  RS_ERR_DEVICE = 4,       /* a HIP runtime call failed                                  */
  RS_ERR_SINGULAR = 5,     /* a diagonal block stayed singular after the pivot guard     */
  RS_ERR_NOCONV = 6,       /* iterative refinement did not reach refine_tol             */
  RS_ERR_OUT_OF_ROOT = 7   /* a node lies outside the fixed root square                   */
} rs_status;

typedef struct {
  double lambda;       /* scalar of (lambda I + K), eq. (biediscretee); -0.5 for the Stokes jump */
  double tol;          /* ID tolerance, relative: a pivot counts while |R_jj| > tol |R_11|     */
  int leaf_size;       /* a box splits while it holds more than leaf_size nodes (Section 2.3)   */
  int n_proxy;         /* points on each box's proxy circle (Section 2.5)                       */
  double proxy_ratio;  /* proxy radius = proxy_ratio * box side                                  */
  double rcond_min;    /* X_RR guard: move a pivot from R to S while rcond_1(X_RR) < rcond_min  */
  int precision;       /* 0 = float64 throughout; 1 = mixed: float32 copies of T, E, F, X_RR^-1
                          (and the border W) serve the solve for every box whose rcond_1(X_RR)
                          is at least mixed_rcond_min (the others keep float64); vectors, sums,
                          the pivoted QR, the inverses and the root stay float64; 2 = float32
                          bulk: as 1, and moreover the entries of M_B and A_BB are computed in
                          float32 from box-local offsets and the Schur-complement products
                          (X_SR, X_RS, X_RR of eq. tmat; E, F, X_SS of eq. schurmat) run on
                          FP32 matrix cores with float32 accumulation; the pivoted QR (rank
                          decision), T, the X_RR inverse with its guard, the root and the
                          refinement residual stay float64.  Its entries carry float32
                          rounding, so its ID tolerance should stay above ~1e-6           */
  double refine_tol;   /* refinement target: max-column ||[f;0] - A x||_2 / ||f||_2             */
  int refine_max;      /* 0: direct solve; > 0: at most this many refinement iterations        */
  int has_root;        /* 1: use root[] as the fixed root square; 0: bounding square of nodes */
  double root[3];      /* fixed root square: centre x, centre y, side                           */
  int solve_graph;     /* 1: refinement iterations replayed as a captured HIP graph, two per
                          launch, with the convergence test on the device (a converged or
                          exhausted iteration leaves x unchanged); 0: launched one by one      */
  double mixed_rcond_min; /* precision 1: smallest rcond_1(X_RR) of a box whose solve reads
                          float copies (float rounding of its factors is then amplified by at
                          most about 1/mixed_rcond_min); > 1 keeps every box in float64     */
  int apply_shape;     /* kernel shape of the exact operator apply (refinement residual):
                          -1 = chosen per (N, ncols) by timing every candidate shape once per
                          process (the autotuner); k >= 0 = candidate k (invalid ones fall
                          back to a fixed default).  Every shape gives bitwise the same result */
  int refine_update;   /* 1 (default): after the first exact float64 residual, the residual of a
                          refinement iteration is updated as r - A dx, with A dx (dx the
                          iteration's correction, small) computed on FP32 matrix cores; its
                          rounding is bounded per node and the bound's norm, accumulated over
                          the updates, is added to the residual norm in the convergence test,
                          so a converged solve is certified against the exact residual; the
                          exact float64 residual is taken again once that sum passes a quarter
                          of refine_tol.  0: every residual is the exact float64 [f;0] - A x */
  int kernel;          /* 0 (default): the Stokes double layer with its augmentation (Section 3.1).
                          1: the Laplace Neumann formulation of Section 4.4.1: u = S mu and
                          f = (lambda I - D + N) mu with D the adjoint double layer
                          -(1/2pi) ((x - y) . n(x)) / |x - y|^2 (normal at the target, pointing
                          out of the domain), N mu = the integral of mu over the boundary and no
                          augmentation (n_holes = 0: every curve_id 0, whatever the number of
                          curves).  The unknown layout stays two per node: unknown 2i is mu at
                          node i, unknown 2i+1 an uncoupled one whose row is lambda x (it joins
                          no box; the solve returns f / lambda there, 0 for 0).  Every
                          precision applies; refinement
                          takes exact residuals (refine_update acts as 0); rs_apply_f32 is not
                          available; rs_evaluate returns (S mu, d(S mu)/dx) per target */
} rs_params;

/* Fill *p with the defaults: lambda -0.5, tol 1e-10, leaf 64, 64 proxy points
 * at 1.5 x side, rcond_min 1e-12, float64, refine_tol 1e-8, refine_max 0
 * (direct solve), no fixed root, solve_graph 1, mixed_rcond_min 1e-4, apply_shape -1,
 * refine_update 1, kernel 0 (Stokes). */
void rs_default_params(rs_params* p);

/* Build the adaptive quadtree (Section 2.3) for a boundary discretisation and
 * copy the geometry to the device.
 *   n_nodes             number of boundary nodes N (> 0)
 *   xy, normal          [N][2] positions and unit normals (|n| = 1 within 1e-12)
 *   weight              [N] quadrature weights (> 0)
 *   curvature           [N] signed curvature (diagonal limit of D)
 *   curve_id            [N] 0 = outer curve, 1..n_holes = hole index
 *   n_holes             p >= 0
 *   hole_xy             [p][2] one interior point c_h per hole (Stokeslet/rotlet
 *                       centre); NULL = centroid of the hole's nodes
 * On success *out receives a new context.  RS_ERR_OUT_OF_ROOT if a fixed
 * root was requested and a node lies outside it. */
rs_status rs_build_tree(const rs_params* prm, int n_nodes, const double* xy,
                        const double* normal, const double* weight,
                        const double* curvature, const int* curve_id, int n_holes,
                        const double* hole_xy, rs_ctx** out);

/* Compute the factorization (Sections 2.2-2.7 with the bordered root of
 * Section 3.2) on the device.  Blocks until the factorization is complete. */
rs_status rs_factor(rs_ctx* ctx);

/* Solve the augmented system for nrhs right-hand sides (eq. kinv, eq. solution).
 *   f             host, (2N) x nrhs, column-major, leading dimension 2N
 *   x             host, (2N + 3p) x nrhs, column-major, leading dimension 2N + 3p
 *   rel_residual  host [nrhs] or NULL: ||[f;0] - A x||_2 / ||f||_2 per column,
 *                 with A applied exactly in float64 on the device
 * With refine_max > 0 the solve is iterative refinement: the residual
 * [f;0] - A x is evaluated exactly in float64 on the device (O(N^2) pairs)
 * and the factorization (with the float32 factor copies when precision = 1)
 * is the inner solver, until every column reaches refine_tol; RS_ERR_NOCONV
 * means refine_max iterations did not reach it, x then holds the last iterate
 * and rel_residual (if given) its residuals. */
rs_status rs_solve(rs_ctx* ctx, int nrhs, const double* f, double* x, double* rel_residual);

/* As rs_solve, with f and x device pointers (same layouts) used on the
 * stream set by rs_set_stream.  The call returns after the solve completed. */
rs_status rs_solve_dev(rs_ctx* ctx, int nrhs, const double* f_dev, double* x_dev);

/* Replace the data of n_moved nodes and update the factorization (Section
 * 2.8): boxes whose unknowns or proxy-disk neighbourhood changed are
 * recompressed, every other box keeps its factors, the root (and the border
 * H, Psi^T) is always redone.  The root square is kept, so the result equals
 * a fresh factorization of the new geometry.
 *   idx                 [n_moved] node indices (distinct, in [0, N))
 *   xy, normal, weight, curvature   new values, [n_moved][2] / [n_moved]
 *   hole_xy             NULL or [p][2] new interior points for all holes
 * RS_ERR_OUT_OF_ROOT if a moved node leaves the root square (nothing is
 * changed then; rebuild the context). */
rs_status rs_update_moved_nodes(rs_ctx* ctx, int n_moved, const int* idx, const double* xy,
                                const double* normal, const double* weight,
                                const double* curvature, const double* hole_xy);

/* Factor n contexts together (the many-geometry batch): level by level, the
 * boxes of all contexts are compressed by one launch per kernel (Section 2.7's
 * level parallelism extended across geometries; the paper's Scheme A runs
 * independent factorizations side by side).  The contexts must live on one
 * device and share lambda, tol, n_proxy, proxy_ratio, rcond_min and
 * precision; the first context's stream is used.  Each context ends up exactly
 * as after its own rs_factor.  On failure every context is left unfactored
 * and carries the message. */
rs_status rs_factor_batch(rs_ctx** ctxs, int n);

/* Update after curves were inserted or deleted (Section 2.8's updating applied
 * to the experiment of Section 4.2, where holes are added to and removed from
 * the domain): the context receives a whole new boundary, in the arrays and
 * conventions of rs_build_tree (N and p may both change), and old_of_new[j],
 * the old index of new node j or -1 for a node that did not exist.  Kept nodes
 * keep their relative order and their data (position, normal, weight,
 * curvature), else RS_ERR_ARG.  The context's root square is kept
 * (RS_ERR_OUT_OF_ROOT if a node lies outside it).  Boxes whose compression
 * inputs are unchanged keep their factors; the others, and the root with H
 * and Psi^T for the new set of holes, are recomputed.  The result equals a
 * fresh factorization of the new boundary with the same root.  RS_ERR_STATE
 * before rs_factor.  Argument errors leave the context as it was; any later
 * failure leaves it unfactored. */
rs_status rs_update_geometry(rs_ctx* ctx, int n_nodes, const double* xy, const double* normal,
                             const double* weight, const double* curvature, const int* curve_id,
                             int n_holes, const double* hole_xy, const int* old_of_new);

/* rs_update_moved_nodes for n contexts together (the related geometries of one
 * finite-difference step of a shape optimization, Section 4's Scheme A): every
 * context's nodes are moved, then the boxes that need recompression in all
 * contexts share one launch per kernel and level.  Entry i of each array
 * holds context i's arguments with the meaning of rs_update_moved_nodes;
 * hole_xy may be NULL (no context moves its hole points) or hold NULL
 * entries.  The contexts must satisfy rs_factor_batch's conditions.  All
 * inputs are checked before anything changes: on a bad input nothing is
 * modified and the first bad context's status is returned (its message in
 * that context).  Each context ends up bitwise as after its own update. */
rs_status rs_update_moved_nodes_batch(rs_ctx** ctxs, int n, const int* n_moved, const int* const* idx,
                                      const double* const* xy, const double* const* normal,
                                      const double* const* weight, const double* const* curvature,
                                      const double* const* hole_xy);

/* rs_solve_dev for each of n factored contexts (f_dev[i], x_dev[i] laid out
 * as for rs_solve_dev of context i).  Refined solves with solve_graph = 1 are
 * interleaved: every context's first graph launch is queued before the first
 * wait.  Returns the first non-RS_OK status (each context carries its message). */
rs_status rs_solve_batch(rs_ctx** ctxs, int n, int nrhs, const double* const* f_dev,
                         double* const* x_dev);

/* Use the given hipStream_t (as void*) for all later device work; NULL = the
 * default stream.  The caller keeps the stream alive while the context uses it. */
rs_status rs_set_stream(rs_ctx* ctx, void* hip_stream);

/* Summary of the last factorization (host-side numbers). */
typedef struct {
  int n_nodes, n_holes, n_levels, n_boxes;
  int root_skeleton;          /* |S| at the root                                   */
  int max_box_unknowns;       /* largest active set of a compressed box            */
  int max_rank;               /* largest skeleton                                  */
  int guard_bumps;            /* pivots moved from R to S by the X_RR guard        */
  long long factor_bytes;     /* bytes of factors read by one solve (T, E, F, X_RR^-1) */
  double flops_id;            /* algorithmic flops of the IDs: per box the pivoted QR of M_B
                                 stopped at rank k plus T, 4mnk - 2(m+n)k^2 + (4/3)k^3 + k^2 r */
  double flops_elim;          /* algorithmic flops of the eliminations             */
  double ms_factor;           /* wall time of the last rs_factor                   */
  double ms_solve;            /* wall time of the last rs_solve / rs_solve_dev     */
  int refine_iters;           /* refinement iterations of the last mixed solve     */
  double ms_update;           /* wall time of the last rs_update_moved_nodes       */
  int boxes_recomputed;       /* boxes recompressed by the last update             */
  int apply_config;           /* operator-apply kernel shape in use (autotuner)    */
  double apply_ms;            /* its measured time per apply (0 if not tuned)      */
  int shape_trials;           /* launches of the last factorization that timed a
                                 candidate workgroup count per box (cooperative QR or
                                 elimination); the count never changes a result    */
} rs_stats;
rs_status rs_get_stats(const rs_ctx* ctx, rs_stats* out);

/* Forget every launch shape the process has tuned: the operator-apply kernel
 * shape per (N, columns) and the workgroups per box of the cooperative QR and
 * elimination per level signature.  Later calls tune again from scratch (the
 * shapes never change a result, only the speed).  Must not run while another
 * thread factors, solves or applies with any context. */
void rs_reset_tuning(void);

/* Per-box structure of the factorization, boxes in breadth-first order
 * (root first).  For each box: level, active unknown count n and rank k
 * (k = n for the root, -1 for a box without active unknowns), and its
 * square (centre x, centre y, side) in box_geom[3*i..3*i+2].  Any output
 * pointer may be NULL.  cap = capacity of the arrays in boxes; the number of
 * boxes is returned in *n_boxes (RS_ERR_ARG if cap is too small). */
rs_status rs_get_boxes(const rs_ctx* ctx, int cap, int* n_boxes, int* level, int* n_active,
                       int* rank, double* box_geom);

/* Skeleton unknowns (global unknown indices, in pivot order) of box `box`
 * (breadth-first index).  cap = capacity of `out`; *len receives k. */
rs_status rs_get_skeleton(const rs_ctx* ctx, int box, int cap, int* out, int* len);

/* Apply the augmented operator exactly in float64 on the device:
 * y = A x, x host (2N+3p) x ncols column-major, y host same shape.  This is
 * the residual kernel used by refinement, exposed for verification. */
rs_status rs_apply(rs_ctx* ctx, int ncols, const double* x, double* y);

/* The float32 image of the same operator, as refinement uses it for the
 * image A dx of a correction (rs_params.refine_update): the double-layer pair
 * sums on FP32 matrix cores with float32 accumulation over tiles of 64 sources,
 * the O(N) terms in float64.  x, y as for rs_apply.  bound (nullable, host,
 * N x ncols column-major) receives per node and column a bound on |y - A x| for
 * both of the node's rows (the Psi^T rows are exact up to float64 rounding).
 * RS_ERR_ARG if two distinct nodes are closer than the kernel's float32 range
 * (about 3e-8). */
rs_status rs_apply_f32(rs_ctx* ctx, int ncols, const double* x, double* y, double* bound);

/* Apply the factored inverse to general right-hand sides of the augmented
 * system (eq. kinv with the partitioned root solve of eq. partition): x =
 * A_RS^{-1} b, where b may have nonzero border rows (its last 3p rows are the
 * border right-hand side; the Krylov and refinement vectors of an outer
 * iteration are such vectors).  b, x: host, (2N+3p) x ncols column-major.
 * Uses the factor copies the solve uses (float32 ones for precision 1).
 * RS_ERR_STATE before rs_factor; RS_ERR_ARG for NULL pointers, ncols <= 0 or a
 * non-finite b. */
rs_status rs_apply_inverse(rs_ctx* ctx, int ncols, const double* b, double* x);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the exact
 * operator apply of rs_apply, y = A x, that allocates nothing.  x_dev, y_dev:
 * device pointers, (2N+3p) x ncols column-major, owned by the caller; the
 * work is enqueued on the context's stream and the call returns without
 * waiting (y_dev is valid once the stream reaches that point).  Every
 * intermediate (row-layout copies of x and y, the partial sums of the pair
 * sums) lives in one fixed device array of 8 Mi doubles (64 MiB) that the
 * library holds per device until the process ends; the call fails with
 * RS_ERR_ARG, touching nothing, when what it needs exceeds that: two copies of
 * (2N+3p) x ncols plus the partial sums, one 2N x ncols block per source
 * chunk (48 chunks at 12288 nodes; the message states the need).  The
 * 12288-node, 8-hole workload fits up to 6 columns.
 * The apply shape is the one the autotuner chose for (N, ncols) earlier in
 * the process, else the default one (every shape gives bitwise the same y).
 * All calls on one device share that array: calls that overlap in time on
 * one device (other streams, other contexts, other host threads) race and
 * must be serialised by the caller.  Nothing in the array needs to start at
 * zero. */
rs_status rs_apply_dev_noalloc(rs_ctx* ctx, int ncols, const double* x_dev, double* y_dev);

/* Velocity u(t) = (D mu)(t) + (H lambda)(t) at n_targets points t off the
 * boundary (eq. forwardeq): the double layer of the density by the boundary
 * quadrature plus the Stokeslet and rotlet of every hole.  targets_xy: host,
 * n_targets x 2 (x, y pairs); x: host, (2N + 3p) x ncols column-major, a
 * solution [mu; lambda] as returned by rs_solve; u: host, (2 n_targets) x ncols
 * column-major, rows 2t and 2t + 1 = the x and y components at target t.
 * Plain quadrature: accurate a few node spacings away from the boundary (no
 * near-boundary correction).  Needs only rs_build_tree (no factorization).
 * With kernel 1 (Laplace Neumann, Section 4.4.1) row 2t is the potential
 * u(t) = (S mu)(t) = -(1/2pi) sum_j log|t - y_j| w_j mu_j and row 2t + 1 its
 * x-derivative (the quantity the section's objective measures at the
 * domain's centre). */
rs_status rs_evaluate(rs_ctx* ctx, int n_targets, const double* targets_xy, int ncols, const double* x,
                      double* u);

/* Inverse of a dense n x n matrix by the blocked Gauss-Jordan elimination with
 * partial pivoting that inverts the root system Z (the partitioned root solve
 * of eq. (partition)), on the context's device and stream.  a: host, row-major,
 * finite (RS_ERR_ARG otherwise), not modified; ainv: host, row-major, n x n,
 * written only on success.  RS_ERR_SINGULAR when a pivot column has no nonzero
 * candidate.  Device scratch is allocated and freed inside the call. */
rs_status rs_dense_inverse(rs_ctx* ctx, int n, const double* a, double* ainv);

/* Per-kernel device time, measured with HIP events recorded around every
 * launch on the context's stream while timing is enabled (it adds two event
 * records per launch; disabled by default). */
typedef struct {
  char name[32];       /* kernel family, e.g. "cpqr", "eliminate", "sweep" */
  int launches;
  double total_ms;
} rs_kernel_time;
/* enable: 0 off, 1 per kernel family, 2 per family and tree level ("cpqr@L7"),
 * 3 the pivoted-QR family ("cpqr") only, with no host-phase timers (the least
 * overhead, for timing a run while reporting that family's device time), 4
 * the exact operator apply ("apply_operator") only; in mode 4 refinement
 * iterations are launched one by one instead of as a captured graph, so that
 * every apply is bracketed by events. */
rs_status rs_set_kernel_timing(rs_ctx* ctx, int enable);
/* Copies up to cap entries accumulated since the last reset; *n receives the
 * number of kernel families.  reset != 0 clears the accumulators afterwards. */
rs_status rs_get_kernel_times(rs_ctx* ctx, int cap, rs_kernel_time* out, int* n, int reset);

void rs_destroy(rs_ctx* ctx);

/* Message of the last failed call on ctx (or of the last failed rs_build_tree
 * when ctx is NULL).  Valid until the next call on that context. */
const char* rs_last_error(const rs_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* RS_MI355X_H */
