// Host-visible launch interface between the C ABI and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rs_types.hpp"

namespace rs {

// Per-stage element count of the leaf solve's scratch (K, k, P, Psi).
constexpr int scratch_per_stage(int nx, int nu) { return nu * nx + nu + nx * nx + nx; }
// Matrix-core leaves also keep V and L of Alg. 4 (leaf solve by a forward
// sweep on the stored preliminary solution).
constexpr int scratch_per_stage_fwd(int nx, int nu) { return 2 * nu * nx + nu + 2 * nx * nx + nx; }

typedef hipError_t (*Launcher)(const GroupArgs &, int grid, hipStream_t);

// Kernel kinds, also the index of the per-kind timers of a plan.
enum KernelKind {
    KK_INIT = 0,
    KK_LEAF_UP = 1, KK_TREE = 2, KK_LEAF_DOWN = 3,          // fused solve
    KK_F_LEAF_UP = 4, KK_F_TREE = 5, KK_F_LEAF_DOWN = 6,    // rs_factor
    KK_S_LEAF_UP = 7, KK_S_TREE = 8, KK_S_LEAF_DOWN = 9,    // rs_solve
    KK_RESIDUAL = 10, KK_UPDATE = 11, KK_CHECK = 12,        // mixed-precision refinement
    KK_REPORT = 13,                                         // K norm of the report
    KK_COUNT = 16
};

struct ShapeEntry {
    int nx, nu;
    bool large;              // no fused kernels: the FP64 solve runs on the stored factorization
    bool lb;                 // the stored factorization uses the large-block kernels (global workspace)
    Launcher fp64[3];        // fused: leaf up, tree, leaf down
    Launcher factor[3][3];   // stored factorization [fp64, fp32, bf16-product leaves][pass] (nullptr: none)
    Launcher vsolve[2][3];   // right-hand-side passes on the stored factorization
    Launcher refine[2];      // FP64 residual, refinement update
    int scratch_per_stage;
};

Launcher mfma_factor(int nx, int nu, int which, bool fp32);
Launcher vector_solve(int nx, int nu, int which, bool fp32);
Launcher refine_kernel(int nx, int nu, int which);       // 0 residual, 1 update
Launcher leaf_forward(int nx, int nu);                   // leaf solve on the stored leaf records
// mode 0 also clears active[0 .. nactive); mode 1 counts the instances still
// iterating into *active.
hipError_t launch_refine_check(const InstInfo *tab, int count, const double *part, double *stats, int32_t *conv,
                               int32_t *info, const DevProb *probs, int mode, double tol, int32_t *active,
                               int nactive, int with_knorm, hipStream_t st);
// Finite-input check (RS_PLAN_CHECK_INPUTS): per leaf, the smallest
// offending place per instance into first[] (preset to INT32_MAX), then
// RS_ERR_ARG and the place in the status words.
hipError_t launch_scan(const GroupArgs &g, int32_t *first, hipStream_t st);
hipError_t launch_scan_mark(int count, const int32_t *first, int32_t *info, hipStream_t st);
// KKT-matrix infinity norm of each leaf's rows (PART_KN of the leaf parts).
hipError_t launch_knorm(const GroupArgs &g, hipStream_t st);
// rs_info records (40 bytes each) from the statistics (or nullptr) and the
// status words.
hipError_t launch_report(int count, const double *stats, const int32_t *info, int refined, void *out,
                         hipStream_t st);

// Large-block family (any n_x, n_u up to 128): stored factorization with a
// per-workgroup workspace of large_unit_bytes.
constexpr int LB_LEAF_UNITS = 2048, LB_TREE_UNITS = 256;
bool large_shape(int nx, int nu);
size_t large_unit_bytes(int nx, int nu);
Launcher large_factor(int which, bool fp32, bool bf16 = false);
Launcher large_vector(int which, bool fp32);
Launcher large_refine(int which);
Launcher mfma_factor_leaf32(int nx, int nu, int which);   // FP32 leaves of n_x = 64 (which 0 up, 2 down)

const ShapeEntry *find_shape(int nx, int nu);

// Device scratch of rs_batch_solve_noalloc (rs_static.hip): its device
// address on the current device (taken once per device), and its size.
constexpr size_t STATIC_SCRATCH_BYTES = size_t(64) << 20;
void *static_scratch(size_t *bytes);
hipError_t launch_init(int32_t *info, int count, int32_t *queues, int nq, hipStream_t st);
hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t st);
// padded copies of the inputs of npad instances (back = false), or their w
// copied back to the caller (back = true)
hipError_t launch_pad(const PadArgs *args, int npad, bool back, hipStream_t st);

}  // namespace rs
