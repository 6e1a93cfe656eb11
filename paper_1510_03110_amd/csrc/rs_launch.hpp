// Host-visible launch interface between the C ABI and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rs_types.hpp"

namespace rs {

// Per-stage element count of the leaf solve's scratch (K, k, P, Psi).
constexpr int scratch_per_stage(int nx, int nu) { return nu * nx + nu + nx * nx + nx; }

typedef hipError_t (*Launcher)(const GroupArgs &, int grid, hipStream_t);

// Kernel kinds, also the index of the per-kind timers of a plan.
enum KernelKind { KK_INIT = 0, KK_LEAF_UP = 1, KK_TREE = 2, KK_LEAF_DOWN = 3, KK_COUNT = 8 };

struct ShapeEntry {
    int nx, nu;
    Launcher fp64[3];        // leaf up, tree, leaf down
    int scratch_per_stage;
};

const ShapeEntry *find_shape(int nx, int nu);
hipError_t launch_init(int32_t *info, int count, int32_t *queues, int nq, hipStream_t st);
hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t st);

}  // namespace rs
