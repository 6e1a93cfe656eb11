/*
 * rs.h - C ABI of the parallel Riccati Newton-step solver for MI355X (gfx950).
 *
 * The library solves the unconstrained finite-time optimal control problem
 * P(N) of Nielsen & Axehill, "An O(log N) Parallel Algorithm for Newton Step
 * Computations with Applications to Moving Horizon Estimation" (Sec. 2,
 * eq. "org_eqc_problem"):
 *
 *   minimise  sum_{t=0}^{N-1} ( 1/2 [x_t;w_t]' [[Qx_t, Qxw_t],[Qxw_t', Qw_t]] [x_t;w_t]
 *                               + lx_t' x_t + lw_t' w_t + c_t )
 *             + 1/2 x_N' QxN x_N + lN' x_N + cN
 *   subject to x_0 = x0,  x_{t+1} = A_t x_t + B_t w_t + a_t,  t = 0..N-1,
 *
 * i.e. one Newton step (KKT solve) of an interior-point or active-set method
 * for MHE.  It returns the primal solution (x, w), the dual variables
 * lam_t = P_t x_t - Psi_t (Alg. 3) and the optimal value.
 *
 * Method (Sec. 4-5): the horizon is split into subintervals ("leaves") that
 * are reduced independently by Alg. 4; the reduced master problem is reduced
 * again up a tree of depth O(log N) (Alg. 5), the top problem is solved and
 * the solution is propagated back down (Alg. 6).  The result is exact (non-
 * iterative): it equals the serial Riccati solution up to rounding.
 *
 * Conventions for every entry point:
 *  - All problem and solution pointers are DEVICE pointers to FP64 data.
 *    Matrices are row-major; block t of an array of r-by-c blocks starts at
 *    element t*stride (stride in elements; stride 0 = the same block for
 *    every stage, e.g. time-invariant A).  Vectors are dense row-major
 *    arrays (N*nx means element [t*nx + i]).
 *  - The caller owns every buffer, including the workspace.  The library
 *    never allocates device memory on the solve path; plan creation
 *    allocates a small pinned host staging area only.
 *  - Calls are asynchronous on the given stream (a hipStream_t passed as
 *    void*, NULL = the default stream).  The return value reports argument
 *    and launch errors only.  Numerical failures are written per instance
 *    into the optional device array info_dev[2*count]:
 *        info_dev[2*i]   = rs_status of instance i (RS_OK, RS_ERR_NOT_SPD,
 *                          RS_ERR_SINGULAR_MASTER, RS_ERR_NOT_CONVERGED)
 *        info_dev[2*i+1] = failing stage index (or -1)
 *    and are valid once the stream has reached the end of the call.
 *  - No exception crosses the ABI.  A plan must not be used by two calls in
 *    flight at the same time (its workspace holds the tree's state).
 */
#ifndef RS_H
#define RS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum rs_status {
    RS_OK = 0,
    RS_ERR_ARG = 1,              /* invalid argument (dims, NULL pointer, size)      */
    RS_ERR_NOT_SPD = 2,          /* G_{t+1} not positive definite (Alg. 1 assumes it) */
    RS_ERR_SINGULAR_MASTER = 3,  /* reduced G of a master stage singular (Sec. 4.2)  */
    RS_ERR_NOT_CONVERGED = 4,    /* mixed precision: refinement missed the target    */
    RS_ERR_NOMEM = 5,            /* workspace smaller than rs_plan_workspace_size     */
    RS_ERR_HIP = 6,              /* a HIP runtime call failed                         */
    RS_ERR_UNSUPPORTED = 7       /* (nx, nu) has no compiled kernel, or bad option    */
} rs_status;

typedef enum rs_precision {
    RS_FP64 = 0,        /* every step in FP64                                         */
    RS_MIXED_FP32 = 1,  /* leaf Riccati in FP32, master levels and the KKT residual
                           in FP64, iterative refinement to the requested tolerance  */
    RS_MIXED_BF16 = 2   /* as RS_MIXED_FP32, with the products P [A B], A'PA, A'PB
                           and B'PB of the leaf stages on BF16 matrix cores (FP32
                           accumulation); shapes served by the large-block kernels
                           only (RS_ERR_UNSUPPORTED otherwise); max_refine default 20 */
} rs_precision;

/* rs_problem.flags: the instance is left untouched by this call (its outputs
 * and status are not written).  A serving loop keeps one plan over all its
 * sessions and marks the sessions without a pending request this way. */
#define RS_PROB_SKIP 1

/* One instance of P(N).  Matrices and vectors: device pointers, FP64. */
typedef struct rs_problem {
    int32_t nx, nu, N;
    int32_t flags;                    /* RS_PROB_SKIP: exclude the instance from this call */
    /* stage matrices, N blocks each (RHS independent) */
    const double *Qx;  int64_t sQx;   /* nx*nx blocks, Q_{x,t}                       */
    const double *Qw;  int64_t sQw;   /* nu*nu blocks, Q_{w,t}, positive definite      */
    const double *Qxw; int64_t sQxw;  /* nx*nu blocks, Q_{xw,t}; NULL = zero           */
    const double *A;   int64_t sA;    /* nx*nx blocks                                  */
    const double *B;   int64_t sB;    /* nx*nu blocks                                  */
    const double *QxN;                /* nx*nx terminal weight Q_{x,N}                 */
    /* right-hand side */
    const double *x0;                 /* nx, initial state xbar_0                      */
    const double *a;                  /* N blocks of nx (stride sa): affine term a_t; NULL = zero */
    const double *lx;                 /* N blocks of nx (stride slx): l_{x,t}; NULL = zero */
    const double *lw;                 /* N blocks of nu (stride slw): l_{w,t}; NULL = zero */
    const double *c;                  /* N constants c_t (stride sc); NULL = zero      */
    const double *lN;                 /* nx terminal linear cost l_N; NULL = zero      */
    const double *cN;                 /* 1 terminal constant; NULL = zero              */
    /* solution (written) */
    double *x;                        /* (N+1)*nx states x_0..x_N                       */
    double *w;                        /* N*nu inputs / process noise w_0..w_{N-1}       */
    double *lam;                      /* (N+1)*nx duals lam_0..lam_N                    */
    double *obj;                      /* 1 optimal value; NULL = not wanted            */
    /* element strides between the stages of a, lx, lw and c (dense arrays:
     * nx, nx, nu, 1; 0 = the same vector every stage).  With strides a
     * window may live in stage-major records, as a serving ring does. */
    int64_t sa, slx, slw, sc;
} rs_problem;

typedef struct rs_options {
    int32_t precision;   /* rs_precision                                              */
    int32_t Ns;          /* leaf (subinterval) length N_s >= 1; 0 = library default    */
    int32_t branch;      /* master stages per master subproblem (>= 2); 0 = default    */
    int32_t max_refine;  /* mixed precision: maximum refinement steps; 0 = default 5  */
    double tol;          /* mixed precision: relative KKT residual target; 0 = 1e-10  */
    int32_t flags;       /* RS_PLAN_* bits                                            */
    int32_t leaf_chunk;  /* > 0: FP64 plans of large-block shapes process their leaves
                            in chunks of this many and keep the factorization of one
                            chunk only (see below); 0 = the whole factorization     */
} rs_options;

/* rs_options.leaf_chunk (Alg. 6 at k = 0 solves every leaf subproblem again
 * with its parent's message, so a leaf's factorization need not outlive its
 * reduction): the workspace holds the stored factorization of at most
 * leaf_chunk consecutive leaves (in plan order) instead of all of them; every
 * chunk is factored on the way up (reduction, Alg. 4) and factored again on
 * the way down (solve), twice the leaf matrix work for a factor store that no
 * longer grows with the batch.  rs_batch_solve only (rs_factor / rs_solve:
 * RS_ERR_ARG); FP64 plans whose every shape runs on the large-block kernels
 * (else RS_ERR_UNSUPPORTED at plan creation); with RS_PLAN_REPORT the
 * residual and backward error are reported, est_fwd_err is -1. */

/* rs_options.flags: reserve workspace for the stored factorization so that
 * rs_factor / rs_solve can be used (about (4 nx^2 + 4 nu^2 + 2 nu nx) doubles
 * per stage more).  Implied by RS_MIXED_FP32. */
#define RS_PLAN_FACTORED 1

/* rs_options.flags: rank-revealing master stages (Sec. 4.2, the reduction
 * with a basis U_1 of range(S'), eqs. Bh_def and Gh_Hh_def).  Every reduced
 * subproblem's M = S Qbar^{-1} S' is factored by Cholesky with diagonal
 * pivoting, M = B B' up to the rank n_uo = rank(S'), stopped once the
 * largest remaining pivot is at most n_x eps max_i M_ii (eps of the
 * precision M was formed in); the master stage takes that B (n_x x n_x, zero
 * columns after n_uo) as its input matrix and the identity as its input
 * weight.  It has the same B Q_w^{-1} B' = M as the U_1 stage, hence the same
 * master solution, and a positive definite G_hat also when Ns*nu < nx (then
 * allowed, down to Ns = 1) or when a subinterval's inputs leave some state
 * directions unreached.  Costs one n_x^3 / 3 factorization per leaf and per
 * master subproblem.  A receding-horizon plan reuses stored M1 messages only
 * from calls with the same flag. */
#define RS_PLAN_RANK_REVEAL 2

/* rs_options.flags: per-instance report of every solve (rs_info, read with
 * rs_info_report).  The quantities are those of the KKT system of P(N)
 * (Sec. 3: the optimality conditions whose solution the Newton step is;
 * unknowns lam_0, x_0, w_0, lam_1, ..., x_N, right-hand side r), in infinity
 * norms and FP64:
 *   rel_resid   = ||r - K z|| / ||r||                 (returned solution z)
 *   bwd_err     = ||r - K z|| / (||K|| ||z|| + ||r||) (normwise backward error)
 *   est_fwd_err = estimated ||z - z*|| / ||z*||
 * FP64 plans: after the solve, one FP64 residual pass gives rel_resid and
 * bwd_err, and one correction solve K d = r - K z with the plan's own kernels
 * (measured, not applied) gives est_fwd_err = ||d|| / ||z|| (about twice the
 * solve's time in all).  Mixed plans: rel_resid and est_fwd_err are those of
 * the refinement (see rs_refine_stats); bwd_err is formed from the final
 * residual.  Either way ||K|| comes from one extra pass over the stage
 * matrices per factorization.  Without this flag rs_info_report gives the
 * status words, and for mixed plans rel_resid, est_fwd_err and the
 * refinement count, with bwd_err = -1 (FP64 plans: all three measures -1). */
#define RS_PLAN_REPORT 4

/* rs_options.flags: check the inputs for NaN and infinity on the device after
 * every call (one more pass over them).  An instance with a non-finite entry
 * in any of its input arrays gets status RS_ERR_ARG in info_dev, whatever
 * the solve reported, and as stage the first offending place: -1 for x0,
 * t for the data of stage t (Qx, Qw, Qxw, A, B, a, lx, lw, c), N for the
 * terminal data (QxN, lN, cN).  Its outputs are not meaningful. */
#define RS_PLAN_CHECK_INPUTS 8

/* rs_options.flags: tile shape.  Instances with n_x = 16 or 32 and n_u < 16
 * are by default solved on the 16 x 16 matrix-core tile kernels with their
 * inputs padded to n_u = 16 (inputs that act on nothing, see the padding
 * kernels); with this flag they run on the kernels for their own shape
 * instead (wavefront and large-block kernels).  An autotuner chooses. */
#define RS_PLAN_NATIVE_TILES 16

/* rs_options.flags: down pass of the master levels of the stored
 * factorization (rs_factor / rs_solve, mixed precision, and every solve of
 * the shapes that run on the large-block kernels).  By default every master
 * subproblem below the top is solved on the way down
 * by a forward sweep on the records of its own reduction (Alg. 4 keeps
 * P, K, V, L_t and the preliminary Psi, k of each master stage; with the
 * terminal costate lam_N sent by the parent, w = K x + k + L_t lam_N and
 * lam = P x - Psi + V lam_N), the superposition that the leaf solve also
 * uses: the master levels are factored once.  With this flag the down pass
 * factors every such subproblem again from its parent's message (P, Psi;
 * Alg. 6 as the paper states it), twice the master-level matrix work; kept
 * for comparison.  Both give the same solution up to rounding. */
#define RS_PLAN_REFACTOR_DOWN 32

/* Per-instance result report (device memory, 40 bytes each). */
typedef struct rs_info {
    double rel_resid;       /* ||r - K z||_inf / ||r||_inf                          */
    double bwd_err;         /* ||r - K z||_inf / (||K||_inf ||z||_inf + ||r||_inf)  */
    double est_fwd_err;     /* estimated relative forward error of z                */
    int32_t refine_iters;   /* corrections applied (mixed precision; 0 in FP64)    */
    int32_t bad_stage;      /* failing stage index, or -1                           */
    int32_t status;         /* rs_status of the instance                            */
    int32_t reserved;
} rs_info;

typedef struct rs_plan_s *rs_plan;

/*
 * Build the tree plan (Alg. 5/6 levels, leaves, work lists) for a batch of
 * `count` instances whose shapes are dims[3*i+0..2] = (nx, nu, N).  Host only:
 * nothing is launched.  Errors: RS_ERR_ARG (count < 1, nx < 1, nu < 1, N < 1,
 * Ns*nu < nx for a multi-leaf instance without RS_PLAN_RANK_REVEAL, which
 * would make the reduced input weight singular, Sec. 4.2 remark),
 * RS_ERR_UNSUPPORTED (no kernel for a shape/precision).
 */
rs_status rs_plan_create(int32_t count, const int32_t *dims, const rs_options *opt,
                         rs_plan *plan_out);

/*
 * As rs_plan_create, with a leaf length and branch per instance: dims5 holds
 * (nx, nu, N, Ns, branch) per instance, Ns = 0 / branch = 0 taking the
 * plan-wide value of opt.  The tree of an instance depends only on its own
 * row, never on the rest of the batch, so an instance gives bit-identical
 * results alone and in any batch (an autotuner chooses Ns and branch per
 * (nx, nu, N range, precision)).  Errors as rs_plan_create.
 */
rs_status rs_plan_create_ex(int32_t count, const int32_t *dims5, const rs_options *opt,
                            rs_plan *plan_out);

/*
 * Plan with subintervals and master groups of chosen sizes (Sec. 4.1: the
 * subintervals i = 0..p need not have equal lengths N_i; Alg. 5: each level's
 * master problem is split into batches of any size).  For instance i,
 * dims[3*i+0..2] = (nx, nu, N); its leaf lengths, in stage order, are
 * leaf_len[leaf_off[i] .. leaf_off[i+1]) (each >= 1, summing to N; the last
 * leaf carries the terminal cost); its master group sizes for levels 1, 2,
 * ... are branch[branch_off[i] .. branch_off[i+1]) (each >= 2, at least one;
 * the last repeats for deeper levels, and a level with at most that many
 * stages is the top problem).  leaf_off and branch_off have count + 1
 * entries.  opt.Ns and opt.branch are not used.  Host only.  Errors as
 * rs_plan_create, and RS_ERR_ARG when the lengths do not sum to N, a length
 * or group size is out of range, or, without RS_PLAN_RANK_REVEAL, a leaf
 * other than the last has length * nu < nx.
 */
rs_status rs_plan_create_split(int32_t count, const int32_t *dims, const int32_t *leaf_off,
                               const int32_t *leaf_len, const int32_t *branch_off,
                               const int32_t *branch, const rs_options *opt, rs_plan *plan_out);

/*
 * Receding-horizon plan (serving): dims8 holds per instance
 *   (nx, nu, N, Ns, branch, start, reuse_lo, reuse_hi)
 * where `start` >= 0 is the absolute index of the window's first stage.  The
 * leaves are laid out on absolute stage boundaries (multiples of Ns, as in
 * the subinterval split of Sec. 4.1): the first leaf runs from `start` to the
 * second boundary after it (the first if `start` is on a boundary), so every
 * leaf but the last keeps at least Ns stages; then full interior leaves
 * a = [a Ns, (a+1) Ns); the last leaf ends with the window and carries the
 * terminal cost.  The stored factorization of interior leaf a lives in ring
 * block a mod (N / Ns + 1) of its instance, at a place in the workspace that
 * depends only on (nx, nu, N, Ns) of the instances in order, so consecutive
 * plans with the same instance list share one workspace and its factors.
 * Interior leaves with reuse_lo <= a < reuse_hi are not factored again: their
 * stored factors and reduced form (Alg. 4 output) from an earlier call on the
 * same workspace are used.  The caller guarantees that the stage matrices of
 * those leaves are unchanged since that call; after a call with window start
 * s, the leaves a in [first_end / Ns, (s + N - 1) / Ns) hold current factors,
 * with first_end = (s / Ns + (s % Ns == 0 ? 1 : 2)) Ns (integer division;
 * none if s + N <= first_end).  The vector passes and the master levels run
 * in full on every call; the FP64 solve always uses the stored factorization.
 * Errors as rs_plan_create, and RS_ERR_ARG for start < 0.
 */
rs_status rs_plan_create_ring(int32_t count, const int32_t *dims8, const rs_options *opt,
                              rs_plan *plan_out);

/*
 * Move a receding-horizon plan to new window positions and reuse ranges
 * (dims8 as for rs_plan_create_ring, with the same (nx, nu, N, Ns, branch)
 * rows): its tables are rebuilt on the host and uploaded by the next call;
 * pinned buffers, events and the bound workspace are kept, so a serving loop
 * neither allocates nor frees host memory per request.  Must not be called
 * while a call on the plan is still to be queued by another thread.
 * Errors: RS_ERR_ARG (not a receding-horizon plan, or rows whose shapes,
 * horizons or leaf lengths differ from the plan's), as rs_plan_create_ring.
 */
rs_status rs_plan_ring_update(rs_plan plan, const int32_t *dims8);

/*
 * MHE front-end (Sec. 2, eq. org_mhe): one moving-horizon estimation problem
 * with samples k = 0..Nmhe, device pointers, FP64, row-major blocks, element
 * strides between samples (0 = the same block for every sample):
 *   x_{k+1} = A_k x_k + B_k w_k + a_k,  y_k = C_k x_k + v_k + d_k,
 * (w_k, v_k) with nominal values (wtil_k, vtil_k) and joint covariance
 * [[Qw_k, Qwv_k], [Qwv_k', Qv_k]], x_0 with estimate xtil0 and covariance Ptil0.
 * The process noise has the state dimension (n_w = n_x).
 */
typedef struct rs_mhe {
    int32_t nx, ny, Nmhe;
    int32_t nw;                          /* process noise dimension; 0 = nx          */
    const double *A;    int64_t sA;      /* nx*nx                                  */
    const double *B;    int64_t sB;      /* nx*nw noise input matrix                */
    const double *a;    int64_t sa;      /* nx; NULL = zero                        */
    const double *C;    int64_t sC;      /* ny*nx                                  */
    const double *d;    int64_t sd;      /* ny; NULL = zero                        */
    const double *y;    int64_t sy;      /* ny measurements                        */
    const double *wtil; int64_t swtil;   /* nw; NULL = zero                        */
    const double *vtil; int64_t svtil;   /* ny; NULL = zero                        */
    const double *Qw;   int64_t sQw;     /* nw*nw process noise covariance, SPD     */
    const double *Qv;   int64_t sQv;     /* ny*ny measurement noise covariance      */
    const double *Qwv;  int64_t sQwv;    /* nw*ny cross covariance; NULL = zero     */
    const double *xtil0;                 /* nx                                     */
    const double *Ptil0;                 /* nx*nx, SPD                             */
} rs_mhe;

/*
 * Write the UFTOC problem P(N), N = Nmhe + 2, of each MHE problem into the
 * arrays named by out[i] (Sec. 2: the state x_{-1} = xtil0 and the noise
 * w_{-1} = x_0 - xtil0 are prepended and time is shifted by one; stage 0 holds
 * the arrival cost with Q_w = Ptil0^{-1}, stage k + 1 the cost of sample k with
 * the inverse joint noise covariance; zero terminal cost).  Written: Qx, Qw,
 * Qxw (if non-NULL), A, B (blocks of out[i]'s strides), a, lx, lw, c, QxN,
 * lN, cN and x0 (= xtil0), through out[i]'s pointers; out[i].nx = nx,
 * out[i].nu = max(nx, nw), out[i].N = Nmhe + 2.  The stage-0 noise has nx
 * components and the samples' nw, so every stage's input is padded to
 * max(nx, nw) with inputs that act on nothing (zero columns of B and Qxw,
 * an identity block of Qw, zero lw); they come out zero in the solution.
 * The result is then solved with rs_batch_solve; x_t of the solution is the
 * estimate of x_{t-1} and w_{t} (t >= 1, first nw components) the noise
 * estimate of sample t - 1.  Asynchronous on `stream`.  nx <= 48 and
 * nw + ny <= 48.  A covariance that is not
 * positive definite sets info_dev[2i] = RS_ERR_NOT_SPD, info_dev[2i+1] = k
 * (-1 for Ptil0) when info_dev is given.  Errors: RS_ERR_ARG (sizes, NULL
 * required pointers, Qwv without an out.Qxw array).
 */
rs_status rs_mhe_to_uftoc(int32_t count, const rs_mhe *mhe, const rs_problem *out, void *stream,
                          int32_t *info_dev);

/*
 * Interior-point kernels for P(N) with input bounds wlo_t <= w_t <= whi_t (the
 * inequality-constrained MHE problem whose Newton steps P(N) gives, Sec. 3).
 * A primal-dual iteration (Mehrotra predictor-corrector) is, on the caller's
 * stream: rs_ip_newton(phase 0) [residuals, Q_w + Sigma, Newton right-hand
 * side; stats[0..4] = max |r_x|, max |r_w|, max |r_l| (and |x_0 - xbar_0|),
 * sum of slack * multiplier, number of finite bounds], rs_factor and rs_solve
 * on `newton` (a plan with RS_PLAN_FACTORED), rs_ip_step(phase 0) [stats[5],
 * stats[6] = largest primal / dual step in (0, 1]], rs_ip_mu [stats[7] =
 * complementarity at the affine step], rs_ip_newton(phase 1, sigma mu)
 * [corrector right-hand side], rs_solve, rs_ip_step(phase 1, sigma mu),
 * rs_ip_update.  All arrays are device FP64, stage-major and dense (stride
 * nu for the bounds unless 0).  `newton` describes the Newton system: the
 * problem's Qx, Qxw, A, B, QxN; its own Qw (N nu*nu, written), a, lx, lw, c,
 * lN, x0 (written) and x, w, lam (the step, written by rs_solve).
 */
typedef struct rs_ip {
    int32_t nx, nu, N, reserved;     /* nx, nu <= 64                                    */
    rs_problem prob;                 /* P(N); its x, w, lam hold the current iterate    */
    const double *wlo; int64_t swlo; /* N blocks of nu: lower bounds (<= -1e300: none)  */
    const double *whi; int64_t swhi; /* upper bounds (>= 1e300: none)                   */
    double *ml, *mu;                 /* N nu multipliers of the lower / upper bounds    */
    rs_problem newton;               /* the Newton system (see above)                   */
    double *dw_aff, *dml, *dmu;      /* N nu: affine input step, multiplier steps       */
    double *part;                    /* (N + 1) * 8 per-stage partial results           */
    double *stats;                   /* 8 results (see above)                           */
} rs_ip;

rs_status rs_ip_newton(const rs_ip *ip, int32_t phase, double sigma_mu, void *stream);
rs_status rs_ip_step(const rs_ip *ip, int32_t phase, double sigma_mu, void *stream);
rs_status rs_ip_mu(const rs_ip *ip, double alpha_p, double alpha_d, void *stream);
rs_status rs_ip_update(const rs_ip *ip, double alpha_p, double alpha_d, void *stream);

/*
 * Write the per-instance report of the last rs_batch_solve / rs_solve with
 * this plan and workspace into report_dev[count] (device memory, rs_info
 * records), asynchronously on `stream`, after that call on the same stream.
 * info_dev: the status array passed to that call (NULL if it was NULL).  The
 * measures are meaningful for instances with status RS_OK; see
 * RS_PLAN_REPORT for what is formed with and without it.  Errors: RS_ERR_ARG
 * (NULL plan, work or report_dev, unaligned work), RS_ERR_HIP.
 */
rs_status rs_info_report(rs_plan plan, const void *work, const int32_t *info_dev, rs_info *report_dev,
                         void *stream);

/* Device workspace bytes the plan needs (caller allocates, 256-byte aligned). */
rs_status rs_plan_workspace_size(rs_plan plan, size_t *bytes);

rs_status rs_plan_destroy(rs_plan plan);

/*
 * Fused Newton-step solve of all `count` instances: Alg. 4/5 up the tree,
 * Alg. 1-3 on the top problem, Alg. 6 back down.  probs is a HOST array of
 * `count` descriptors (device pointers inside) with the shapes given at plan
 * creation.  In RS_MIXED_FP32 plans this performs factor + solve + FP64
 * residual refinement (see rs_solve).  Returns RS_ERR_NOMEM if work_bytes is
 * too small, RS_ERR_ARG for a NULL pointer or a shape mismatch.
 */
rs_status rs_batch_solve(rs_plan plan, const rs_problem *probs, void *work,
                         size_t work_bytes, void *stream, int32_t *info_dev);

/*
 * rs_batch_solve for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the workspace is a device array of RS_NOALLOC_SCRATCH_BYTES (64 MiB) that
 * the library holds on every GPU it runs on from its load until the process
 * ends, so the caller passes only the problems (inputs and outputs, as for
 * rs_batch_solve), the stream and the optional status array.  The call
 * allocates nothing (no hipMalloc, hipFree, pinned or library allocation):
 * the plan's pinned staging is taken at plan creation.  Every call on one GPU
 * shares that GPU's array, which keeps the last call's contents; each call
 * binds it afresh (tables, descriptors, cleared tree flags), so calls that
 * follow one another on the GPU are independent, but calls that overlap on
 * one GPU (other streams, other threads) race and must not be issued.
 * The plan's kernel timing is not recorded by this call.  Results are the
 * same as rs_batch_solve's.  Errors: RS_ERR_NOMEM if the plan's workspace
 * (rs_plan_workspace_size) exceeds RS_NOALLOC_SCRATCH_BYTES, RS_ERR_ARG for
 * receding-horizon plans (their stored factors cannot live in a shared
 * array) and as rs_batch_solve, RS_ERR_HIP if the plan was created without
 * a device.
 */
#define RS_NOALLOC_SCRATCH_BYTES (((size_t)64) << 20)
rs_status rs_batch_solve_noalloc(rs_plan plan, const rs_problem *probs, void *stream, int32_t *info_dev);

/*
 * Factorization part only (Alg. 1 and the matrix lines of Alg. 4 on every
 * level, including the down-pass factorizations with the true terminal
 * weights).  Reads the matrix fields of probs (Qx, Qw, Qxw, A, B, QxN);
 * stores every factor in the workspace: per stage P_t, L^{-1} and L^{-T}
 * (G_{t+1} = L L'), K_{t+1} and, for Alg. 4, V_t.  Numerical failures
 * (RS_ERR_NOT_SPD with the stage, RS_ERR_SINGULAR_MASTER) go to info_dev as
 * for rs_batch_solve.  The factors stay valid until the next rs_factor or
 * rs_batch_solve with the same plan and workspace.  Needs a plan created
 * with RS_PLAN_FACTORED or a mixed precision (else RS_ERR_ARG); every shape
 * that rs_plan_create accepts has factor kernels (matrix-core kernels for the
 * tile shapes, large-block kernels for the others).
 */
rs_status rs_factor(rs_plan plan, const rs_problem *probs, void *work, size_t work_bytes,
                    void *stream, int32_t *info_dev);

/*
 * Solve part only (Alg. 2-3 and the vector lines of Alg. 4): uses the factors
 * stored by the last rs_factor with the same plan and workspace, reads the
 * right-hand side fields (x0, a, lx, lw, c, lN, cN) and A, B, QxN of probs
 * and writes x, w, lam and obj.  The matrices must be unchanged since
 * rs_factor.  Several rs_solve calls may follow one rs_factor (iterative
 * refinement, predictor-corrector steps).  The status words in info_dev are
 * left as rs_factor wrote them (a solve adds only a tree-wait failure).
 * For RS_MIXED_FP32 plans the FP32 factors are refined in FP64 to the
 * plan's tolerance: info_dev reports RS_ERR_NOT_CONVERGED on failure.
 */
rs_status rs_solve(rs_plan plan, const rs_problem *probs, void *work, size_t work_bytes,
                   void *stream, int32_t *info_dev);

/* Plan introspection: key 0 = number of leaves, 1 = number of tree work items,
 * 2 = maximum tree depth (levels above the leaves), 3 = leaf length Ns,
 * 4 = branch, 5 = precision, 6 = refinement iterations launched by the last
 * mixed-precision call (converged instances skip the remaining ones; the
 * per-instance count is in rs_refine_stats). */
int64_t rs_plan_query(rs_plan plan, int32_t key);

/* Export the plan's work tables for host-side inspection (tests, tooling).
 * what = 0: one row of 7 int64 per leaf (instance, first stage, length,
 *           flags: 1 = holds the terminal cost, 2 = is the whole problem,
 *           level-1 slot, scratch offset, shape group);
 * what = 1: one row of 11 int64 per tree item (kind: 0 reduce, 1 eliminate
 *           last, 2 top solve, 3 down solve; instance, level, first slot,
 *           stage count, holds-terminal, terminal slot, output slot, first
 *           dependency, dependency count, shape group).
 * Writes only if cap_rows is large enough; returns the row count (-1 on a
 * bad argument).  Host only. */
int64_t rs_plan_export(rs_plan plan, int32_t what, int64_t *out, int64_t cap_rows);

/* Kernel timing (measurement aid).  While enabled, each call records a pair
 * of HIP events on its stream around every kernel it launches.
 * rs_plan_kernel_times waits for the recorded events and returns, per kernel
 * kind, the summed elapsed milliseconds and the number of launches since the
 * last reset; reset != 0 starts a new window.  Kinds: 0 status/queue reset;
 * fused solve 1 leaf reduction, 2 tree levels, 3 leaf solve; rs_factor
 * 4 leaf, 5 tree, 6 leaf down; rs_solve 7 leaf, 8 tree, 9 leaf down;
 * refinement 10 FP64 residual, 11 update, 12 convergence check;
 * 13..15 reserved.  ms and launches point to RS_KERNEL_KINDS host values. */
#define RS_KERNEL_KINDS 16
rs_status rs_plan_set_timing(rs_plan plan, int32_t enable);
rs_status rs_plan_kernel_times(rs_plan plan, double *ms, int64_t *launches, int32_t reset);

/* Refinement statistics of the last mixed-precision solve with this plan and
 * workspace, 5 doubles per instance, copied to host memory `out` (waits for
 * `stream`):
 *   [0] relative KKT residual ||r - K z||_inf / ||r||_inf of the returned
 *       solution, evaluated in FP64;
 *   [1] estimated relative forward error: d_k (d_k / d_{k-1}), where d_k is
 *       the last correction relative to the solution (max over the x, w, lam
 *       blocks) and d_{k-1} the one before (1 for the first);
 *   [2] corrections applied;  [3] converged flag;  [4] d_k.
 * An instance stops refining once a correction has been applied, [0] <= tol
 * and [1] <= tol/10; it is reported RS_ERR_NOT_CONVERGED if that does not
 * happen within max_refine corrections.  RS_ERR_ARG for a
 * plan that is not RS_MIXED_FP32. */
rs_status rs_refine_stats(rs_plan plan, const void *work, double *out, void *stream);

/*
 * HIP graph of one call (mode 0 = rs_batch_solve, 1 = rs_factor, 2 =
 * rs_solve): binds the descriptors as the call would, then captures its whole
 * kernel sequence on `stream` (which must not be the NULL stream) into an
 * executable graph.  Nothing runs at creation except the descriptor upload.
 * rs_graph_launch replays the call on any stream: the launch overhead of the
 * multi-kernel sequence (mixed precision: up to 6 + 7*max_refine kernels) is
 * paid once.  A replay reads the problem descriptors bound most recently to
 * the plan's workspace, so data may change behind the same pointers between
 * replays; new pointers need a new graph.  The graph clears the tree's
 * completion flags with a kernel at its start.  One graph of a plan may run
 * at a time, and not concurrently with a direct call on the same workspace.
 */
typedef struct rs_graph_s *rs_graph;
rs_status rs_graph_create(rs_plan plan, int32_t mode, const rs_problem *probs, void *work,
                          size_t work_bytes, void *stream, int32_t *info_dev, rs_graph *graph_out);
rs_status rs_graph_launch(rs_graph graph, void *stream);
rs_status rs_graph_destroy(rs_graph graph);

const char *rs_status_string(rs_status s);

#ifdef __cplusplus
}
#endif

#endif /* RS_H */
