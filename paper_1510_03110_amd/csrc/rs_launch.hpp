// Host-visible launch interface between the C ABI and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rs_types.hpp"

namespace rs {

// Per-stage element count of the leaf solve's scratch (K, k, P, Psi).
constexpr int scratch_per_stage(int nx, int nu) { return nu * nx + nu + nx * nx + nx; }

typedef hipError_t (*GroupLauncher)(const GroupArgs &, int tree_grid, hipStream_t);

struct ShapeEntry {
    int nx, nu;
    GroupLauncher fp64;
    int scratch_per_stage;
};

const ShapeEntry *find_shape(int nx, int nu);
hipError_t launch_init(int32_t *info, int count, int32_t *queues, int nq, hipStream_t st);
hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t st);

}  // namespace rs
