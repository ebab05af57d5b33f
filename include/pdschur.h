/*
 * pdschur.h -- C ABI of the MI355X (gfx950) hot path of localized-collision
 * Projective Dynamics (Wang, Tao, Brandt, Cutting, Sifakis: "Optimized
 * Processing of Localized Collisions in Projective Dynamics", SCA 2020).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every call returns pd_status (PD_OK = 0).  No C++ exception crosses the
 *   ABI.  A failed call leaves a message retrievable with pd_last_error().
 * - "dev" pointers are device memory owned by the caller (contiguous, float64
 *   unless stated).  "host" pointers are host memory read during the call.
 * - Vectors over nodes are coordinate-major: [3][len] (all x, then all y,
 *   then all z).  Global arrays have len = n_nodes; region arrays have len = m.
 * - Region-local index = rank of the node among the collision-prone free
 *   nodes in ascending global id.
 * - Work is enqueued on the HIP stream given to pd_schur_build.  Calls return
 *   after enqueueing, except pd_schur_build and a pd_global_solve with a
 *   non-NULL info pointer, which synchronize the stream.
 * - Invalid sizes or NULL pointers -> PD_ERR_INVALID with no side effect.  A
 *   HIP runtime failure -> PD_ERR_HIP and the context refuses further work.
 * - A context is not thread-safe; calls on one context must not overlap.
 */
#ifndef PDSCHUR_H
#define PDSCHUR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pd_ctx pd_ctx;

typedef enum {
  PD_OK = 0,
  PD_ERR_INVALID = -1,     /* bad argument; nothing was enqueued */
  PD_ERR_HIP = -2,         /* HIP runtime error (sticky) */
  PD_ERR_OOM = -3,         /* device allocation failed */
  PD_ERR_NOT_SPD = -4,     /* non-positive pivot in a Cholesky factorization */
  PD_ERR_IR_STALLED = -5,  /* iterative refinement did not reach its tolerance */
  PD_ERR_STATE = -6        /* call order violated (e.g. backsub before condense) */
} pd_status;

typedef enum {
  PD_FP64 = 0,     /* FP64 factor and solve */
  PD_FP32_IR = 1,  /* FP32 factor, refinement with an FP64 residual */
  PD_BF16_IR = 2   /* BF16-operand / FP32-accumulate factor, FP64-residual refinement */
} pd_precision;

/* Tetrahedral mesh and partition (Sec. 3.2 and Sec. 4.2 of the paper). */
typedef struct {
  int64_t n_nodes;
  int64_t n_tets;
  const double *rest;       /* host [3][n_nodes] rest positions */
  const int32_t *tets;      /* host [4][n_tets] vertex ids, det(D_m) > 0 required */
  const uint8_t *region;    /* host [n_nodes] 1 = collision-prone node (x2) */
  const uint8_t *dirichlet; /* host [n_nodes] 1 = prescribed node (not an unknown) */
  double mu;                /* shear modulus; lambda is dropped (Sec. 3.2) */
  double density;           /* backward Euler: mass per unit rest volume (dt > 0) */
  double dt;                /* backward-Euler time step; 0 = quasistatic (Sec. 3.2) */
  double mu_prime;          /* biphasic material (Sec. 5.3): stiffness of the strain */
  double sigma_min;         /*   limit mu' ||F - Q||^2, Q = F with its singular values */
  double sigma_max;         /*   clamped to [sigma_min, sigma_max]; mu_prime = 0: off */
  int32_t interior_order;   /* interior factor (Sec. 4.3): 0 = breadth-first levels from
                               x2, eliminated level by level; 1 = nested dissection,
                               factored supernode by supernode (multifrontal) */
  int32_t nd_leaf;          /* nested dissection: largest part not bisected further
                               (0: 256); ignored for interior_order = 0 */
} pd_mesh;

typedef struct {
  int32_t ir_iters;      /* refinement steps taken (0 for PD_FP64) */
  int32_t bad_pivot;     /* 1-based index of the first non-positive pivot, else 0 */
  int32_t fell_back;     /* 1 if the call refactored in FP64 after a stall */
  int32_t reserved;
  double rel_residual;   /* max over x,y,z of ||g - (S+P)u|| / ||g|| (FP64) */
} pd_solve_info;

/* Builds everything that stays constant while the mesh deforms (Sec. 4.3,
 * eq. par_chol and eq. k22 without collisions):
 *  - element shape operators and volumes, the scalar stiffness K
 *    (one of the three identical coordinate blocks, Sec. 3.2);
 *  - the partition: x2 = region & !dirichlet, x1 = other free nodes,
 *    E_beta = tets with all four vertices in x2, E_alpha = the rest (Sec. 4.5);
 *  - the interior factor (dense FP64 on the GPU): with interior_order = 0, x1
 *    is ordered by breadth-first distance from x2 and eliminated level by
 *    level (Z_k = S_k^-1 kept per level); with interior_order = 1, by
 *    geometric nested dissection (pd_nd_analyse) and factored supernode by
 *    supernode, keeping X_s = L_ss^-1 and L_Bs per supernode;
 *  - the dense Schur complement S = K22 - K21 K11^-1 K12 (m x m, FP64).
 * Synchronous.  *out receives a context freed by pd_destroy.
 * Errors: PD_ERR_INVALID for out-of-range vertex ids, an empty region or a
 * non-positive rest volume, interior_order outside {0, 1} or nd_leaf outside
 * [0, 8192]; PD_ERR_NOT_SPD if an interior level block or supernode is not
 * positive definite (e.g. an interior component with no Dirichlet node). */
pd_status pd_schur_build(const pd_mesh *mesh, void *hip_stream, pd_ctx **out);

/* Sizes: m = |x2|, n1 = |x1|, E_beta and E_alpha tet counts, interior levels
 * (nested dissection: the height of the supernode tree, the number of
 * batched steps of each sweep). */
pd_status pd_query(const pd_ctx *ctx, int64_t *m, int64_t *n1, int64_t *n_beta,
                   int64_t *n_alpha, int64_t *n_levels);

/* host [m] <- global ids of the region nodes in region-local order. */
pd_status pd_region_nodes(const pd_ctx *ctx, int32_t *ids);

/* dev [m][m] column-major <- S (both triangles).  Enqueued copy. */
pd_status pd_get_schur(pd_ctx *ctx, double *S);

/* dev x2 [3][m] <- positions of the region nodes taken from x [3][n_nodes]. */
pd_status pd_region_gather(pd_ctx *ctx, const double *x, double *x2);

/* Local step and forces on E_alpha (Alg. 1 steps 1-2): R_e = polar(F_e(x))
 * (Sec. 3.2, orthogonal Procrustes, det R = +1), P = 2 mu (F - R) and
 * f = -sum_e Vol_e P B_e on every node.  x, f: dev [3][n_nodes]; R_alpha:
 * dev [9][n_alpha] row-major 3x3 per tet (FP64, or FP32 with rot_fp32) or
 * NULL.  rot_fp32 = 1: the polar decomposition (and the biphasic projection)
 * in FP32 from the rounded F, forces accumulated in FP64.  Forces on
 * Dirichlet nodes are written too (they are not used by the solve). */
pd_status pd_local_step_full(pd_ctx *ctx, const double *x, void *R_alpha, double *f,
                             int rot_fp32);

/* Backward Euler (mesh.dt > 0; Sec. 3.2 states that PD applies to implicit
 * backward Euler as it does to the quasistatic problem): each step minimises
 * 1/(2 dt^2) (x - y)^T M (x - y) + E(x) with lumped masses M (a quarter of
 * density * Vol_e to each node of tet e) and the inertial target
 * y = x_n + dt v_n.  pd_schur_build then adds D = M / dt^2 to the constant
 * matrix (so to S and the interior factor), and pd_local_step_full adds the
 * inertia force -D (x - y) on every free node.  This call sets the target y
 * (dev [3][n_nodes], caller-owned, read by every later pd_local_step_full;
 * NULL clears it).  PD_ERR_STATE for a quasistatic context; with dynamics,
 * pd_local_step_full returns PD_ERR_STATE while no target is set. */
pd_status pd_set_inertia_target(pd_ctx *ctx, const double *y);

/* End of a backward-Euler step (all dev [3][n_nodes]): v = (x - x_prev) / dt,
 * then x_prev = x and y = x + dt v (the next step's target).  PD_ERR_STATE for
 * a quasistatic context. */
pd_status pd_time_step_advance(pd_ctx *ctx, const double *x, double *x_prev, double *v,
                               double *y);

/* Forward substitution through the interior factor (Alg. 1 step 3;
 * Sec. 4.4 Step 1): y2 = f2 - A21 A11^-1 f1, with f taken from f [3][n_nodes].
 * y2: dev [3][m].  Keeps A11^-1 f1 in the context for pd_backsub. */
pd_status pd_condense_rhs(pd_ctx *ctx, const double *f, double *y2);

/* Collision detection against rigid spheres for conforming proxies (paper
 * Sec. 3.3).  A proxy (region-local node id prox[j]) is in collision iff
 * ||p - c_s|| < r_s; its target is c_s + r_s (p - c_s)/||p - c_s|| (+z at
 * the centre); the deepest sphere wins, ties to the lowest index.
 * Writes one penalty per proxy in the fixed-width layout of
 * pd_collision_update: idx [n_prox][8] (slot 0 = prox[j], others -1),
 * w [n_prox][8], c [n_prox] (k or 0 when free), t [3][n_prox].
 * prox: dev int32 [n_prox]; spheres: dev [4][n_sph] (cx, cy, cz, r). */
pd_status pd_detect_spheres(pd_ctx *ctx, int32_t n_prox, const int32_t *prox,
                            int32_t n_sph, const double *spheres, double k,
                            const double *x2, int32_t *idx, double *w, double *c,
                            double *t);

/* Self-contact detection for paired region nodes (two lips of a slit):
 * pair j = (pairs[j], pairs[n_pairs + j]) = (lower-lip node a, upper-lip
 * node b), region-local, dev int32 [2][n_pairs].  The pair is in collision
 * iff z_b < z_a (the lips interpenetrate); it then becomes a zero-rest-length
 * spring between the two nodes (Sec. 3.3 with the proxy and the surface point
 * both on the mesh): W row [1, -1] on (a, b), target 0, stiffness k.  Output
 * layout as pd_detect_spheres, one penalty per pair (c = 0 when apart). */
pd_status pd_detect_pairs(pd_ctx *ctx, int32_t n_pairs, const int32_t *pairs, double k,
                          const double *x2, int32_t *idx, double *w, double *c, double *t);

/* Embedded (non-conforming) proxies (Sec. 3.3, eq. p_j_v): a proxy moves
 * with the tetrahedron that contains its rest position, p = sum_k w_k x_k
 * over that tet's four nodes.  For each point pts[:, j] (dev [3][n_pts]) this
 * finds the lowest-index candidate tet (cand: dev int32 [4][n_cand],
 * region-local node ids; positions pos: dev [3][m], e.g. the region's rest
 * positions) whose four barycentric coordinates are all >= -1e-12, and
 * writes tet[j] (dev int32 [n_pts]), its nodes eidx[j][0..3] (dev int32
 * [n_pts][4]) and the coordinates ew[j][0..3] (dev [n_pts][4]); a point in
 * no candidate gets tet -1, nodes -1 and weights 0.  Candidates with a node
 * outside 0..m-1 are skipped. */
pd_status pd_embed_points(pd_ctx *ctx, int32_t n_pts, const double *pts, int32_t n_cand,
                          const int32_t *cand, const double *pos, int32_t *tet, int32_t *eidx,
                          double *ew);

/* Sphere detection (the rule of pd_detect_spheres) for embedded proxies
 * given by eidx/ew as written by pd_embed_points: p_j = sum_k ew[j][k]
 * x2[eidx[j][k]]; penalty j's W row is the proxy's four weights (slots 0..3;
 * slots 4..7 unused), target on the sphere, c = k when inside.  A proxy with
 * a node outside 0..m-1 gives an unused row (c = 0).  Output layout as
 * pd_detect_spheres. */
pd_status pd_detect_embedded_spheres(pd_ctx *ctx, int32_t n_prox, const int32_t *eidx,
                                     const double *ew, int32_t n_sph, const double *spheres,
                                     double k, const double *x2, int32_t *idx, double *w,
                                     double *c, double *t);

/* Rest-pose level-set self-collision of embedded proxies (Sec. 5.1, with the
 * penalty of Sec. 3.3).  Bodies: candidate tets cand (dev int32 [4][n_cand],
 * region-local), the rest signed distance of their body at their corners
 * cand_phi (dev [4][n_cand], linear over the tet, < 0 inside) and their body
 * id cand_body (dev int32 [n_cand]); proxy j (eidx/ew as above) belongs to
 * body prox_body[j] (dev int32 [n_prox]).  Per proxy: p = sum w x2; the
 * lowest candidate of another body that contains p in the deformed
 * positions x2 (dev [3][m]), skipping tets that share a node with the
 * proxy's own tet; X = its rest point (rest2: dev [3][m]) with the same
 * barycentric coordinates and phi(X); if phi(X) < 0, the rest surface point
 * X - phi g / |g|^2 (g = grad phi on that tet) is located (same rule) in the
 * rest candidates of the same body, and the penalty is a zero-rest-length
 * spring between the proxy and that point: W row = the proxy's four weights,
 * then minus the surface point's coordinates over its tet's nodes (a node
 * already in the row carries the sum in its slot; at most 8 slots), target
 * 0, c = k.  Otherwise the row holds the proxy's weights and c = 0.  One
 * wavefront per proxy, candidates scanned in index order.  Output layout as
 * pd_detect_spheres. */
pd_status pd_detect_levelset(pd_ctx *ctx, int32_t n_prox, const int32_t *eidx, const double *ew,
                             const int32_t *prox_body, int32_t n_cand, const int32_t *cand,
                             const double *cand_phi, const int32_t *cand_body,
                             const double *rest2, double k, const double *x2, int32_t *idx,
                             double *w, double *c, double *t);

/* Penalty update (Sec. 3.3 eq. E_col_C and Sec. 4.3 eq. k22): stores the
 * penalty set for the next pd_global_solve, whose matrix becomes
 * H = S + W^T C W, and writes f_col = -W^T C (W x2 - t) (dev [3][m]).
 * Penalty j touches up to 8 region nodes idx[j][s] (region-local, -1 =
 * unused, entries within one penalty distinct) with weights w[j][s] and
 * stiffness c[j] >= 0 (0 = inactive); t is dev [3][n_pen].  The arrays are
 * copied; the caller may reuse them after the call.  Marks the factor stale. */
pd_status pd_collision_update(pd_ctx *ctx, int32_t n_pen, const int32_t *idx,
                              const double *w, const double *c, const double *t,
                              const double *x2, double *f_col);

/* Local step on E_beta (Alg. 1 step 4.2, Sec. 4.5) at region positions
 * x2 (dev [3][m]): R_beta (dev [9][n_beta], FP64 or FP32 per rot_fp32, or
 * NULL) and f_beta (dev [3][m]) = forces of the E_beta tets on region nodes. */
pd_status pd_local_step_region(pd_ctx *ctx, const double *x2, void *R_beta,
                               double *f_beta, int rot_fp32);

/* g = ft + f_beta + f_col (Alg. 1 step 4.4), all dev [3][m]; f_beta or f_col
 * may be NULL (treated as zero). */
pd_status pd_assemble_rhs(pd_ctx *ctx, const double *ft, const double *f_beta,
                          const double *f_col, double *g);

/* Dense solve of H u = g with H = S + W^T C W (Alg. 1 steps 4.3 and 4.5,
 * Sec. 4.4 Step 2): refactors H if the penalty set changed (or the precision
 * of the stored factor differs), then solves the three coordinate
 * right-hand sides.  g, u: dev [3][m], g and u must not alias.
 * PD_FP64: FP64 Cholesky and triangular solves.
 * PD_FP32_IR / PD_BF16_IR: the Jacobi-equilibrated D H D is factored in FP32
 * (tile products on FP32 matrix cores, or with BF16 operands and FP32
 * accumulation); that factor preconditions conjugate gradients on H u = g,
 * with H applied in FP64 (the residual g - H u stays FP64), one independent
 * iteration per coordinate column, until max_v ||g_v - H u_v|| / ||g_v|| <=
 * tol (default 1e-8, recomputed from u at the end) or max_steps steps
 * (default 100; see pd_set_refinement).  These modes synchronize the stream
 * once per step.  If the tolerance is not reached, or the low-precision
 * factor meets a non-positive pivot: with fallback on (the default) the call
 * factors H in FP64, solves, and returns PD_OK with info->fell_back = 1; with
 * fallback off it returns PD_ERR_IR_STALLED (PD_ERR_NOT_SPD for the pivot)
 * with u = the last iterate.
 * info (host) may be NULL; when given, the call synchronizes and fills it
 * (ir_iters = conjugate-gradient steps taken).
 * A non-positive pivot of the FP64 factor -> PD_ERR_NOT_SPD (only detected
 * when the call synchronizes, i.e. with info or in the refined modes). */
pd_status pd_global_solve(pd_ctx *ctx, const double *g, double *u, pd_precision prec,
                          pd_solve_info *info);

/* Settings of the refined modes of pd_global_solve: at most max_steps
 * (0..100000) conjugate-gradient steps, relative residual tolerance tol > 0,
 * fallback = 1 to factor in FP64 when the refinement does not reach tol
 * (fell_back reported in pd_solve_info), 0 to return PD_ERR_IR_STALLED.
 * Defaults: 100, 1e-8, 1.  Invalid values -> PD_ERR_INVALID, unchanged. */
pd_status pd_set_refinement(pd_ctx *ctx, int32_t max_steps, double tol, int32_t fallback);

/* FP64 factorization of H = S + W^T C W ahead of the solve (Alg. 1 step 4.3,
 * Sec. 4.4 Step 2), for callers that overlap it with other work: H only
 * depends on the penalty set and S, not on the right-hand side, so the
 * factorization may run on a second stream while pd_backsub, the full local
 * step and pd_condense_rhs of the next iteration run on the first (see
 * pd_use_stream).  n_workgroups > 0 caps the persistent workgroups of the
 * factorization (default 2 per compute unit; fewer leave room for kernels of
 * the other stream); <= 0 keeps the default.
 * overlap_forward = 0: a following pd_global_solve(PD_FP64) runs both
 * triangular solves after the factorization.  overlap_forward = 1: the
 * following pd_global_solve(PD_FP64) may be enqueued on another stream
 * without waiting for the factorization (after this call returns): its
 * forward substitution starts at once and follows the factorization's tile
 * flags row block by row block, and its backward substitution waits for the
 * factorization's end (both through events the library records); nothing
 * else may use the context's factor in between.  The factorization itself
 * never waits for work of another stream (streams may share a hardware
 * queue, which runs in order).  Other values: PD_ERR_INVALID.  A no-op when
 * the factor is current.  Non-positive pivots are reported by a later
 * pd_global_solve with info. */
pd_status pd_factor(pd_ctx *ctx, int32_t n_workgroups, int32_t overlap_forward);

/* Inner update (Alg. 1 steps 4.6-4.7): x2 += u2, delta2 += u2 and
 * ft -= Sigma_alpha u2 with Sigma_alpha = S - A22^(beta).  All dev [3][m]. */
pd_status pd_inner_update(pd_ctx *ctx, const double *u2, double *x2, double *delta2,
                          double *ft);

/* Back substitution (Alg. 1 step 5, Sec. 4.4 Step 3):
 * x1 += A11^-1 (f1 - A12 delta2) using f1 of the last pd_condense_rhs, and
 * x2 += delta2, both written into x (dev [3][n_nodes]).  PD_ERR_STATE if no
 * pd_condense_rhs preceded it. */
pd_status pd_backsub(pd_ctx *ctx, const double *delta2, double *x);

/* ---- Learned warm start (not in the paper) ---------------------------------
 * A three-layer perceptron y = W3 relu(W2 relu(W1 x + b1) + b2) + b3 that
 * predicts the region displacement increment of the next frame from the
 * previous increment and the active-penalty mask.  Products use BF16
 * operands (weights kept as BF16 copies of FP32 master weights; activations
 * and gradients rounded to BF16 when used as operands) with FP32
 * accumulation on the matrix cores.  Loss: sum((y - t)^2) / (2 B n_out).
 * Optimiser: Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected).
 * Parameter packing (host float32): W1 [n_h1][n_in], b1 [n_h1], W2 [n_h2][n_h1],
 * b2 [n_h2], W3 [n_out][n_h2], b3 [n_out] (row-major, concatenated). */
/* ---- Standalone dense FP64 Cholesky -------------------------------------
 * The single-launch dataflow factorization that pd_global_solve / pd_factor
 * apply to H = S + P (Alg. 1 step 4.3; Sec. 4.4 Step 2: one dense Cholesky
 * of the collision-region system per penalty change), for callers that need
 * the factorization of their own SPD matrix. */
typedef struct pd_chol pd_chol;

/* Workspace for matrices of order up to n_max (tile inverses and partial sums
 * 2 x ceil(n_max / 64) x 64 x 64 doubles, ready flags); factorizations are
 * enqueued on hip_stream.  Synchronous.  n_max <= 0 -> PD_ERR_INVALID. */
pd_status pd_chol_create(int64_t n_max, void *hip_stream, pd_chol **out);

/* In place: A dev [n x n] column-major, leading dimension lda (a multiple of
 * 16 doubles, lda >= n; 0 < n <= n_max), A itself aligned to 128 bytes (so
 * that no two 64 x 64 tiles share a cache line; e.g. not an offset view into
 * a larger allocation), symmetric positive definite, lower triangle read.  On return the lower triangle holds L (A = L L^T) and the
 * strictly upper triangle holds L^T.  n_workgroups > 0 caps the persistent
 * workgroups (default two per compute unit).  info_host == NULL: enqueue only.
 * Otherwise the call synchronizes and *info_host receives 0, or the 1-based
 * index of the first non-positive pivot (PD_ERR_NOT_SPD; the reciprocal
 * square root of that pivot is taken as 1 and the factorization runs to the
 * end).  Calls on one handle
 * must not overlap.  Invalid arguments -> PD_ERR_INVALID, nothing enqueued. */
pd_status pd_chol_factor(pd_chol *h, double *A, int64_t lda, int64_t n, int32_t n_workgroups,
                         int32_t *info_host);

/* Waits for the handle's stream and frees the workspace. */
pd_status pd_chol_destroy(pd_chol *h);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * factorization of pd_chol_factor without a handle.  Its workspace is a
 * static device array of the library sized for n <= PD_CHOL_NOALLOC_MAX_N
 * (about 8.1 MB), one copy per GPU, held until the process ends and shared by
 * every call on that GPU: calls that overlap on one GPU (e.g. on two streams)
 * race and must be serialized by the caller.  The first call on a GPU also
 * enqueues a fill that zeroes the array's flags.  Enqueued on hip_stream
 * (the current device's); arguments, layout, result and info_host as for
 * pd_chol_factor.  n > PD_CHOL_NOALLOC_MAX_N -> PD_ERR_INVALID, nothing
 * enqueued.  Calls no allocating routine. */
#define PD_CHOL_NOALLOC_MAX_N 8192
pd_status pd_chol_factor_noalloc(double *A, int64_t lda, int64_t n, int32_t n_workgroups,
                                 void *hip_stream, int32_t *info_host);


/* Schedule of the single-launch dataflow Cholesky (pd_chol_factor, the
 * factorization of H = S + P in pd_global_solve / pd_factor), for checking
 * its index ranges on the host (no GPU work; the kernels decode their
 * tickets with the same code).  For order n (tiles of 64, nt = ceil(n/64)),
 * rhs = 1 when the three right-hand sides ride along as an extra tile row:
 * *ntask receives the number of tasks, and for 0 <= q < *ntask the tile
 * (*i, *j) of ticket q (*i == nt: the right-hand-side row) and *kend, the
 * number of 64-column steps the task accumulates.  n < 1, rhs not 0/1, or q
 * outside [0, *ntask) (q < 0 only queries the count) -> PD_ERR_INVALID. */
pd_status pd_dataflow_task(int64_t n, int32_t rhs, int64_t q, int32_t *i, int32_t *j,
                           int32_t *kend, int64_t *ntask);

/* The nested-dissection ordering and symbolic factorization that
 * pd_schur_build uses for interior_order = 1 (host only, no GPU work;
 * mesh->interior_order is ignored here).  The interior nodes x1 are bisected
 * recursively along the longest side of their bounding box of rest positions
 * at the coordinate change nearest the median; the nodes of one half (the
 * smaller choice) adjacent to the other half form the separator.  Parts of at
 * most leaf nodes, and the separators, are the supernodes, numbered so that
 * every child precedes its parent.
 * sizes (host [3]) <- n1, ns (supernodes), nb (boundary entries).  The
 * arrays, each host memory owned by the caller, are filled when non-NULL:
 *   elim [n1]     node id at each elimination position;
 *   first [ns+1]  supernode s holds positions first[s] .. first[s+1]-1;
 *   parent [ns]   the supernode holding the first key of s's boundary (the
 *                 elimination tree), -1 when that boundary is empty or lies
 *                 in x2 (a root: its update goes to S);
 *   bptr [ns+1], bkey [nb]: boundary of s, ascending keys bkey[bptr[s]..
 *                 bptr[s+1]-1]; a key k < n1 is the elimination position k,
 *                 k >= n1 the region node k - n1 (region-local order).
 * The boundary of s is the set of later nodes coupled to s after the
 * elimination of its subtree: x2 nodes and later x1 nodes adjacent to s, and
 * the boundaries of its children minus s.  Errors: PD_ERR_INVALID for NULL
 * mesh arrays or sizes, out-of-range vertex ids or leaf < 1. */
pd_status pd_nd_analyse(const pd_mesh *mesh, int32_t leaf, int64_t *sizes, int32_t *elim,
                        int32_t *first, int32_t *parent, int64_t *bptr, int32_t *bkey);

typedef struct pd_mlp pd_mlp;

/* Creates the network with the given initial parameters (host, packed as
 * above; initial values are an input, e.g. from a seeded generator).
 * max_batch bounds the batch of every later call.  Synchronous. */
pd_status pd_mlp_create(int32_t n_in, int32_t n_h1, int32_t n_h2, int32_t n_out,
                        int32_t max_batch, const float *params_host, void *hip_stream,
                        pd_mlp **out);

/* host params (packed as above) <- current FP32 master parameters.  Synchronous. */
pd_status pd_mlp_get_params(pd_mlp *mlp, float *params_host);

/* y = network(x): x dev float [batch][n_in], y dev float [batch][n_out]. */
pd_status pd_mlp_forward(pd_mlp *mlp, const float *x, float *y, int32_t batch);

/* One training step on (x, target), both dev float, batch rows.  With
 * grads_host == NULL: forward, backward and an Adam update with rate lr.
 * With grads_host != NULL: the gradients (packed as the parameters) are
 * copied to the host and no update is made.  loss_host (may be NULL)
 * receives the loss before the update; giving it synchronizes. */
pd_status pd_mlp_train_step(pd_mlp *mlp, const float *x, const float *target, int32_t batch,
                            float lr, double *loss_host, float *grads_host);

/* Training batches: dst [B][n_cols] (dev float) <- rows rows[b] (dev int32,
 * each in [0, n_rows)) of src [n_rows][n_cols] (dev float), the first
 * n_scaled columns multiplied by scale (standardisation of increments). */
pd_status pd_mlp_gather_rows(pd_mlp *mlp, const float *src, int32_t n_rows, int32_t n_cols,
                             const int32_t *rows, int32_t B, int32_t n_scaled, float scale,
                             float *dst);

/* *out_host <- mean of |a[i]| over n floats (dev).  Synchronizes. */
pd_status pd_mlp_abs_mean(pd_mlp *mlp, const float *a, int64_t n, double *out_host);

pd_status pd_mlp_destroy(pd_mlp *mlp);

/* Moves the context to another HIP stream (after synchronizing the current
 * one).  Every entry point that does not synchronize (the FP64 path without
 * info, and everything but pd_schur_build, pd_displacement_change and
 * pd_get_timings) only enqueues kernels and device-to-device copies on the
 * stream, so a sequence of them can be captured into a HIP graph and
 * replayed; the dataflow kernels take their epochs from device memory. */
pd_status pd_set_stream(pd_ctx *ctx, void *hip_stream);

/* Moves the context to another HIP stream without synchronizing: later calls
 * enqueue on hip_stream.  The caller orders work across streams (HIP events)
 * and keeps calls that share context state apart: the factorization side
 * (pd_detect_*, pd_collision_update, pd_local_step_region, pd_factor) and the
 * sweep side (pd_backsub, pd_local_step_full, pd_condense_rhs, pd_region_gather)
 * use disjoint context buffers and may run concurrently; pd_assemble_rhs,
 * pd_global_solve and pd_inner_update read the results of both and must be
 * ordered after them. */
pd_status pd_use_stream(pd_ctx *ctx, void *hip_stream);

/* Phases timed by pd_get_timings. */
typedef enum {
  PD_PHASE_LOCAL_FULL = 0,    /* pd_local_step_full */
  PD_PHASE_CONDENSE = 1,      /* pd_condense_rhs */
  PD_PHASE_DETECT = 2,        /* pd_detect_spheres */
  PD_PHASE_COLLISION = 3,     /* pd_collision_update */
  PD_PHASE_LOCAL_REGION = 4,  /* pd_local_step_region */
  PD_PHASE_ASSEMBLE = 5,      /* pd_assemble_rhs */
  PD_PHASE_HBUILD = 6,        /* pd_global_solve: H = S + W^T C W (lower part) */
  PD_PHASE_FACTOR = 7,        /* pd_global_solve: Cholesky factorization of H */
  PD_PHASE_SOLVE = 8,         /* pd_global_solve: triangular solves (+ refinement) */
  PD_PHASE_INNER_UPDATE = 9,  /* pd_inner_update */
  PD_PHASE_BACKSUB = 10,      /* pd_backsub */
  PD_N_PHASES = 11
} pd_phase;

/* Turns per-phase timing on (1) or off (0).  When on, every entry point
 * records a pair of HIP events on the context stream around its work. */
pd_status pd_set_timing(pd_ctx *ctx, int on);

/* Synchronizes the stream and returns, per phase, the summed milliseconds
 * (host ms[PD_N_PHASES]) and the number of timed calls (host counts, may be
 * NULL) since the previous call; then clears the records. */
pd_status pd_get_timings(pd_ctx *ctx, double *ms, int64_t *counts);

/* Warm-start network input for the next frame (float32, dev [4m]):
 * [scale (x2 - x2_prev) (coordinate-major, 3m) ; mask (m)], mask = 1 at the
 * region nodes prox[j] whose penalty stiffness cpen[j] is non-zero (e.g. the
 * c output of pd_detect_spheres at the start of the frame). */
pd_status pd_warmstart_input(pd_ctx *ctx, const double *x2, const double *x2_prev, float scale,
                             int32_t n_prox, const int32_t *prox, const double *cpen,
                             float *out);

/* x[:, region] += scale * d2 for a float32 region increment d2 (dev [3][m]),
 * x dev [3][n_nodes]: applies a predicted displacement to the region nodes. */
pd_status pd_region_add_f32(pd_ctx *ctx, const float *d2, double scale, double *x);

/* A predicted region increment applied with the static response of the
 * interior (Sec. 4.4 Step 3 with a zero interior force): d = scale * d2
 * (d2 float32 dev [3][m]), plus x2_prev1 - x2_prev2 when both are given (dev
 * [3][m]: the previous frame's increment, so that d2 is a correction of it);
 * then x2 += d and x1 -= A11^-1 A12 d, x dev [3][n_nodes].  The interior
 * nodes then sit where the constant system puts them for the moved region,
 * so the next local step sees the prediction everywhere.  Uses the interior
 * factor's sweep; a following pd_backsub needs a new pd_condense_rhs
 * (PD_ERR_STATE otherwise).  Only one of x2_prev1, x2_prev2 given ->
 * PD_ERR_INVALID. */
pd_status pd_warmstart_apply(pd_ctx *ctx, const float *d2, double scale, const double *x2_prev1,
                             const double *x2_prev2, double *x);

/* Training target of the warm-start network in its residual form: out =
 * scale * ((x2 - x2_prev1) - (x2_prev1 - x2_prev2)) (float32 dev [3][m]; all
 * x dev [3][m]), the change of the region increment from one frame to the
 * next. */
pd_status pd_warmstart_target(pd_ctx *ctx, const double *x2, const double *x2_prev1,
                              const double *x2_prev2, float scale, float *out);

/* Convergence measure of an outer iteration: out[0] = ||x - x_prev||_2 and
 * out[1] = ||x - X||_2 over all free nodes (X = rest positions), for the
 * relative-change test ||x_k - x_{k-1}|| / ||x_k - X|| <= tol.  x, x_prev:
 * dev [3][n_nodes]; out: host [2].  Synchronizes. */
pd_status pd_displacement_change(pd_ctx *ctx, const double *x, const double *x_prev,
                                 double *out);

/* Last error message of the context (valid until the next call on it).
 * With ctx = NULL: the message of the last failed pd_schur_build on this thread. */
const char *pd_last_error(const pd_ctx *ctx);

/* Frees every device and host resource of the context. */
pd_status pd_destroy(pd_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* PDSCHUR_H */
