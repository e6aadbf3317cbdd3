// noalloc.hip -- spmd_launch_noalloc: spmd_launch for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc).
//
// The classes that need cross-block scratch (REDUCE_I32: completion ticket,
// epoch and one status word per block; SCAN_I32 and COMPACT_I32: draw
// ticket and one status word per tile) take it from `scratch`, a static
// device array the library holds on every device it runs on, instead of a
// caller workspace.  The array is cut into one region per class, and a
// region is only ever used by launches of its own class: each launch leaves
// its region as its class's next launch expects it (the ticket re-armed,
// the epoch advanced, so stale status words read as unwritten), so a region
// is cleared once, at the device's set-up, and never again.  Classes
// without scratch are launched exactly as by spmd_launch.
//
// The host never uses the name `scratch` as an address: on the host side it
// is a stand-in for the device symbol.  The device address is looked up
// with hipGetSymbolAddress once per device, with that device current, and
// kept in the device's DevInfo.
#include <string.h>

#include "common.hpp"

namespace spmd {

namespace {

constexpr size_t REGION = SPMD_NOALLOC_REGION_BYTES;
constexpr int NREGION = 3;  // REDUCE_I32, SCAN_I32, COMPACT_I32

static __device__ __align__(256) uint8_t scratch[NREGION * REGION];

int region_of(int kernel_id) {
    switch (kernel_id) {
    case SPMD_REDUCE_I32: return 0;
    case SPMD_SCAN_I32: return 1;
    case SPMD_COMPACT_I32: return 2;
    default: return -1;
    }
}

}  // namespace

// Per-device set-up, called by runtime_dev with the device current: the
// device address of this device's copy of the array, cleared once.
int noalloc_setup(uint8_t** out) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e);
    if ((e = hipMemset(p, 0, sizeof(scratch))) != hipSuccess) return hip_fail(e);
    *out = static_cast<uint8_t*>(p);
    return SPMD_OK;
}

}  // namespace spmd

using namespace spmd;

extern "C" int spmd_launch_noalloc(int kernel_id, spmd_dim3 grid, spmd_dim3 block, size_t dyn_shmem, void** args,
                                   void* stream) {
    const int r = region_of(kernel_id);
    if (r < 0) return spmd_launch(kernel_id, grid, block, dyn_shmem, args, stream);
    const char* sig = spmd_kernel_signature(kernel_id);
    const size_t nargs = strlen(sig) - 1;  // the workspace, the class's last parameter, is not passed
    if (!args) return SPMD_ERR_ARGS;
    for (size_t i = 0; i < nargs; ++i)
        if (!args[i]) return SPMD_ERR_ARGS;
    if (!grid.x || !grid.y || !grid.z || !block.x || !block.y || !block.z) return SPMD_ERR_INVALID_DIM;
    if (spmd_workspace_size(kernel_id, grid, block, 0) > REGION) return SPMD_ERR_WORKSPACE;
    const DevInfo* di = nullptr;
    int rc = runtime_dev(&di);
    if (rc) return rc;
    void* ws = di->scratch + (size_t)r * REGION;
    void* packed[8];
    for (size_t i = 0; i < nargs; ++i) packed[i] = args[i];
    packed[nargs] = &ws;
    return spmd_launch(kernel_id, grid, block, dyn_shmem, packed, stream);
}
