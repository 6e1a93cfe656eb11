// Plain structs shared by the host planner and the device kernels of the
// parallel Riccati solver.  No arithmetic lives here.
#pragma once
#include <stdint.h>

namespace rs {

// Status words written by the kernels (values of rs_status in rs.h).
constexpr int32_t STATUS_OK = 0, STATUS_NOT_SPD = 2, STATUS_SINGULAR_MASTER = 3, STATUS_NOT_CONVERGED = 4;

// Device copy of one problem descriptor (pointers are device pointers).
struct DevProb {
    const double *Qx, *Qw, *Qxw, *A, *B, *QxN;
    const double *x0, *a, *lx, *lw, *c, *lN, *cN;
    double *x, *w, *lam, *obj;
    int64_t sQx, sQw, sQxw, sA, sB;
    int64_t sa, slx, slw, sc;       // element strides of the stage vectors
    int32_t nx, nu, N, flags;    // flags: PROB_SKIP leaves the instance untouched
};
constexpr int32_t PROB_SKIP = 1;

// Input padding of one instance (n_u raised to nup with inputs that act on
// nothing): the caller's arrays, the padded copies in the workspace and their
// stage strides (0 where the caller's stride is 0), and the caller's w.
struct PadArgs {
    const double *B, *Qw, *Qxw, *lw;
    int64_t sB, sQw, sQxw, slw;
    double *Bp, *Qwp, *Qxwp, *lwp, *wp;
    int64_t sBp, sQwp, sQxwp, slwp;
    double *w;
    int32_t nx, nu, nup, N, flags, pad_;
};

// One leaf (level-0 subproblem, a batch of original stages, Sec. 4.1).
struct LeafItem {
    int32_t inst;      // instance index
    int32_t t0, len;   // stages t0 .. t0+len-1
    int32_t flags;     // LEAF_LAST: holds the terminal cost; LEAF_TOP: whole problem
    int32_t slot;      // level-1 slot: receives its reduced form (up), holds the
                       // parent's solution for it (down)
    int32_t m1;        // receding-horizon plans: M1 cache block of an interior leaf (-1: none)
    int64_t scratch;   // element offset of its per-stage factor storage
};
// LEAF_REUSE: its stored factorization and reduced form (M1 cache) are
// current; the factorization pass only copies the cached M1 into its slot.
enum { LEAF_LAST = 1, LEAF_TOP = 2, LEAF_REUSE = 4 };

// One master-level work item of the tree (Alg. 5 reduce / Alg. 6 solve).
struct TreeItem {
    int32_t kind;       // ITEM_UP, ITEM_UP_LAST, ITEM_TOP, ITEM_DOWN
    int32_t inst;
    int32_t level;      // tree level of the node (>= 1)
    int32_t first;      // global slot index of its first stage
    int32_t count;      // number of stages
    int32_t last;       // 1 if the node holds its level's terminal cost
    int32_t term_slot;  // global slot of the level's terminal (valid if last)
    int32_t out_slot;   // slot one level up that receives (UP) / supplies (DOWN) its data
    int32_t dep_first;  // first item it waits for
    int32_t dep_count;  // number of consecutive items it waits for
};
enum { ITEM_UP = 0, ITEM_UP_LAST = 1, ITEM_TOP = 2, ITEM_DOWN = 3 };

// Layout of one master-level slot, in doubles, for state dimension n.
//   M1 (sent to the parent, Alg. 5):   Ahat n*n | Qwhat n*n | Qxhat n*n | ahat n | lxhat n | chat 1
//   M2 (sent to a child, Alg. 6):      xhat n | P n*n | Psi n | cbar 1
//   factors of the down pass:          K n*n | k n
//   stored factorization (factor / solve split), master stage of this slot:
//     up pass (Alg. 4):   P_after n*n | L^{-1} n*n | L^{-T} n*n | K n*n | V_after n*n
//     down pass (Alg. 1): L^{-1} n*n | L^{-T} n*n   (its K is the K above)
struct SlotLayout {
    int n;
    __host__ __device__ int A() const { return 0; }
    __host__ __device__ int Qw() const { return n * n; }
    __host__ __device__ int Qx() const { return 2 * n * n; }
    __host__ __device__ int a() const { return 3 * n * n; }
    __host__ __device__ int lx() const { return 3 * n * n + n; }
    __host__ __device__ int c() const { return 3 * n * n + 2 * n; }
    __host__ __device__ int xh() const { return 3 * n * n + 2 * n + 1; }
    __host__ __device__ int P() const { return 3 * n * n + 3 * n + 1; }
    __host__ __device__ int Psi() const { return 4 * n * n + 3 * n + 1; }
    __host__ __device__ int cb() const { return 4 * n * n + 4 * n + 1; }
    __host__ __device__ int K() const { return 4 * n * n + 4 * n + 2; }
    __host__ __device__ int k() const { return 5 * n * n + 4 * n + 2; }
    __host__ __device__ int uP() const { return 5 * n * n + 5 * n + 2; }
    __host__ __device__ int uL() const { return 6 * n * n + 5 * n + 2; }
    __host__ __device__ int uLT() const { return 7 * n * n + 5 * n + 2; }
    __host__ __device__ int uK() const { return 8 * n * n + 5 * n + 2; }
    __host__ __device__ int uV() const { return 9 * n * n + 5 * n + 2; }
    __host__ __device__ int dL() const { return 10 * n * n + 5 * n + 2; }
    __host__ __device__ int dLT() const { return 11 * n * n + 5 * n + 2; }
    // costate at the end of the node's subproblem (its terminal lam_N), sent
    // down by the fused matrix-core tree and by the superposition sweep of the
    // large-block tree (whose up pass then keeps L_t = -G^{-1} B' V in dL)
    __host__ __device__ int lamN() const { return 12 * n * n + 5 * n + 2; }
    __host__ __device__ int size() const { return ((12 * n * n + 6 * n + 2) + 7) & ~7; }
};

// Stored factorization of one leaf stage (factor / solve split), in the
// factor precision (FP64, or FP32 in mixed-precision plans):
//   up record (Alg. 4 or last-leaf elimination):
//       P_after | L^{-1} | L^{-T} | K | V_after | Lt
//   down record (Alg. 1 with the true terminal, whole-problem leaves only):
//       P_after | L^{-1} | L^{-T} | K
// P_after / V_after are the values after the stage (P_t, V_t), L^{-1} is the
// inverse Cholesky factor of G_{t+1}, K = K_{t+1} and Lt = -G^{-1} B' V_{t+1}.
// The vectors of a solve (Psi_t | k_{t+1}, nx + nu doubles per stage: of the
// preliminary solution for multi-leaf instances, of the true one for
// whole-problem leaves) live in a separate FP64 array.
struct LeafRec {
    int nx, nu;
    __host__ __device__ int P() const { return 0; }
    __host__ __device__ int L() const { return nx * nx; }
    __host__ __device__ int LT() const { return nx * nx + nu * nu; }
    __host__ __device__ int K() const { return nx * nx + 2 * nu * nu; }
    __host__ __device__ int V() const { return nx * nx + 2 * nu * nu + nu * nx; }
    __host__ __device__ int Lt() const { return 2 * nx * nx + 2 * nu * nu + nu * nx; }
    __host__ __device__ int up() const { return 2 * nx * nx + 2 * nu * nu + 2 * nu * nx; }
    __host__ __device__ int down() const { return nx * nx + 2 * nu * nu + nu * nx; }
    __host__ __device__ int per_stage() const { return up() + down(); }
    __host__ __device__ int vec() const { return nx + nu; }
};

// Per-instance entry of the refinement tables: the instance's leaves are
// global leaf indices first_leaf .. first_leaf + nleaves - 1.
struct InstInfo {
    int32_t first_leaf, nleaves, nx, nu, N, pad;
};

// Per-leaf partial results of the refinement kernels (doubles):
//   residual: max |r| (right-hand side), max |r - K z|, objective part,
//             max |z| over the leaf's entries of x, w, lam
//   update:   max |dx|, |dw|, |dlam|, max |x|, |w|, |lam| after the update
//   K norm:   largest absolute row sum of the leaf's rows of the KKT matrix
enum { PART_RHS = 0, PART_RES = 1, PART_OBJ = 2, PART_DX = 3, PART_X = 6, PART_ZN = 9, PART_KN = 10, PART_N = 11 };
// Per-instance refinement statistics (doubles): relative residual of the
// returned solution, estimated relative forward error, corrections applied,
// converged flag, size of the last correction relative to the solution,
// normwise backward error ||r - K z|| / (||K|| ||z|| + ||r||) (infinity
// norms; -1 when ||K|| was not formed).
enum { ST_RRES = 0, ST_EST = 1, ST_ITERS = 2, ST_CONV = 3, ST_DZ = 4, ST_BWD = 5, ST_N = 6 };
// The first ST_PUBLIC statistics are what rs_refine_stats exports.
constexpr int ST_PUBLIC = 5;

// Everything a kernel launch of one shape group needs.
struct GroupArgs {
    const DevProb *probs;
    const LeafItem *leaves;
    int32_t nleaves;
    const TreeItem *items;
    int32_t nitems;
    double *slots;
    void *leaf_scratch;     // T-typed per-stage storage of the leaf solve
    int32_t *flags;         // per tree item: epoch when done
    int32_t *queue;         // tree work-queue counter
    int32_t *info;          // per instance: status, stage
    int32_t epoch;
    int32_t sps;            // fused-solve scratch elements per stage (leaf stage index = scratch / sps)
    void *fstore;           // stored factorization of the leaves (LeafRec per stage, double or float)
    double *fvec;           // down-pass vectors of the leaves (nx + nu doubles per stage)
    // mixed-precision refinement (nullptr / 0 otherwise)
    const DevProb *corr;    // correction problems: same matrices, RHS and outputs in the workspace
    const int32_t *conv;    // per instance: 1 once converged (later passes skip it)
    double *part;           // per global leaf: PART_N partial results
    int32_t leaf_base;      // global index of this group's first leaf
    int32_t ntop;           // leaves that are a whole instance (LEAF_TOP)
    const int32_t *active;  // refinement: instances still iterating (0: the pass has nothing to do)
    // large-block kernels: per-workgroup matrix workspace (lbw_unit bytes per
    // workgroup) and the group's dimensions
    void *lbw;
    int64_t lbw_unit;
    int32_t nx, nu;
    // receding-horizon plans: per interior ring block, the matrix part of the
    // leaf's M1 message (A_hat | Q_w_hat | Q_x_hat, 3 n^2 doubles)
    double *m1cache;
    // rank-revealing master stages: an n_x x n_x identity (the master input
    // weight), nullptr for the plain form B = Q_w = Q_w_hat
    const double *ident;
    // refinement update: 1 = only measure the correction and the solution
    // (no z += d), for an error estimate of the returned solution
    int32_t measure_only;
    // leaf-chunked solves: stage index (in the group's leaf stage numbering)
    // of the first record held by the stored factorization of this launch
    int64_t rec_stage0;
    // master levels of the stored factorization: 1 = the down pass of every
    // master subproblem below the top is the superposition sweep on its up
    // records (Alg. 6 without a second factorization), 0 = factored again
    // with the parent's message
    int32_t superpose;
    // first stage of a leaf's records in the stored factorization
    __host__ __device__ int64_t rec_stage(int64_t leaf_scratch) const { return leaf_scratch / sps - rec_stage0; }
};

}  // namespace rs
