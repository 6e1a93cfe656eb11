// Device scratch of the entry point that allocates nothing
// (rs_batch_solve_noalloc): a file-scope device array that serves as the
// plan's workspace.  Every GPU the library runs on holds its own copy from
// the library's load until the process ends.  Host code must not use the
// array's name as an address (in host code it is a stand-in for the device
// symbol): its device address is taken once per device with
// hipGetSymbolAddress and kept, and only that address is handed to kernels
// and copies.
#include <hip/hip_runtime.h>

#include <mutex>

#include "rs_launch.hpp"

namespace rs {

static __device__ __attribute__((aligned(256))) unsigned char scratch[STATIC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void *scratch_ptr[MAX_DEVICES] = {};
}  // namespace

void *static_scratch(size_t *bytes) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        scratch_ptr[dev] = p;
    }
    if (bytes) *bytes = STATIC_SCRATCH_BYTES;
    return scratch_ptr[dev];
}

}  // namespace rs
