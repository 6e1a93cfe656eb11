// Plain structs shared by the host planner and the device kernels of the
// parallel Riccati solver.  No arithmetic lives here.
#pragma once
#include <stdint.h>

namespace rs {

// Device copy of one problem descriptor (pointers are device pointers).
struct DevProb {
    const double *Qx, *Qw, *Qxw, *A, *B, *QxN;
    const double *x0, *a, *lx, *lw, *c, *lN, *cN;
    double *x, *w, *lam, *obj;
    int64_t sQx, sQw, sQxw, sA, sB;
    int32_t nx, nu, N, pad;
};

// One leaf (level-0 subproblem, a batch of original stages, Sec. 4.1).
struct LeafItem {
    int32_t inst;      // instance index
    int32_t t0, len;   // stages t0 .. t0+len-1
    int32_t flags;     // LEAF_LAST: holds the terminal cost; LEAF_TOP: whole problem
    int32_t slot;      // level-1 slot: receives its reduced form (up), holds the
                       // parent's solution for it (down)
    int32_t pad;
    int64_t scratch;   // element offset of its per-stage factor storage
};
enum { LEAF_LAST = 1, LEAF_TOP = 2 };

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
    __host__ __device__ int size() const { return ((12 * n * n + 5 * n + 2) + 7) & ~7; }
};

// Stored factorization of one leaf stage (factor / solve split), doubles:
//   up record (Alg. 4 or last-leaf elimination): P_after | L^{-1} | L^{-T} | K | V_after
//   down record (Alg. 1 with the true terminal):  P_after | L^{-1} | L^{-T} | K
//   down-pass vectors written by the solve:       Psi_after | k
// P_after / V_after are the values after the stage (P_t, V_t), L^{-1} is the
// inverse Cholesky factor of G_{t+1} and K = K_{t+1}.
struct LeafRec {
    int nx, nu;
    __host__ __device__ int P() const { return 0; }
    __host__ __device__ int L() const { return nx * nx; }
    __host__ __device__ int LT() const { return nx * nx + nu * nu; }
    __host__ __device__ int K() const { return nx * nx + 2 * nu * nu; }
    __host__ __device__ int V() const { return nx * nx + 2 * nu * nu + nu * nx; }
    __host__ __device__ int up() const { return 2 * nx * nx + 2 * nu * nu + nu * nx; }
    __host__ __device__ int down() const { return nx * nx + 2 * nu * nu + nu * nx; }
    __host__ __device__ int vec() const { return nx + nu; }
    __host__ __device__ int per_stage() const { return up() + down() + vec(); }
};

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
    double *fstore;         // stored factorization of the leaves (LeafRec per stage)
};

}  // namespace rs
