// k_scan.hip -- SCAN_I32 kernel and launcher.
//
// Workspace: u32 ticket, u32 done, u32 epoch, u32 pad, then one u64 status
// word per tile.  Blocks take tile indices from the ticket in the order
// they start; the last block to finish re-arms ticket and done and advances
// the epoch, which is the tag of the next launch's status words.
#include "cls_scan.hpp"

namespace spmd {

template <int B, int I>
__global__ __launch_bounds__(B) void scan_i32_kernel(const int32_t* __restrict__ x, int32_t* __restrict__ y,
                                                      uint32_t n, uint32_t* ws, uint32_t* err, bool vec) {
    __shared__ ScanLds<B> L;
    __shared__ uint32_t s_tile, s_tag;
    uint64_t* status = reinterpret_cast<uint64_t*>(ws + 4);
    if (threadIdx.x == 0) {
        s_tile = atomic_add_dev(ws + 0, 1u);
        s_tag = __hip_atomic_load(ws + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    const uint32_t tile = s_tile, tag = s_tag;
    scan_tile<B, I>(x, y, n, tile, status, tag, err, vec, L);
    if (threadIdx.x == 0) {
        const uint32_t d = atomic_add_dev(ws + 1, 1u);
        if (d == gridDim.x - 1u) {
            store_release_dev(ws + 0, 0u);
            store_release_dev(ws + 1, 0u);
            store_release_dev(ws + 2, tag + 1u);
        }
    }
}

size_t ws_scan_i32(spmd_dim3 grid, spmd_dim3, uint64_t) { return 16 + 8ull * grid.x; }

template <int B>
static void launch_b(uint32_t I, dim3 g, size_t dyn, hipStream_t s, const int32_t* x, int32_t* y, uint32_t n,
                     uint32_t* ws, uint32_t* err, bool vec) {
    dim3 b(B);
    switch (I) {
    case 1: hipLaunchKernelGGL((scan_i32_kernel<B, 1>), g, b, dyn, s, x, y, n, ws, err, vec); break;
    case 2: hipLaunchKernelGGL((scan_i32_kernel<B, 2>), g, b, dyn, s, x, y, n, ws, err, vec); break;
    case 4: hipLaunchKernelGGL((scan_i32_kernel<B, 4>), g, b, dyn, s, x, y, n, ws, err, vec); break;
    case 8: hipLaunchKernelGGL((scan_i32_kernel<B, 8>), g, b, dyn, s, x, y, n, ws, err, vec); break;
    case 16: hipLaunchKernelGGL((scan_i32_kernel<B, 16>), g, b, dyn, s, x, y, n, ws, err, vec); break;
    case 32: hipLaunchKernelGGL((scan_i32_kernel<B, 32>), g, b, dyn, s, x, y, n, ws, err, vec); break;
    }
}

int launch_scan_i32(const LaunchCtx& c) {
    const uint32_t B = c.block.x;
    if (c.block.y != 1 || c.block.z != 1 || c.grid.y != 1 || c.grid.z != 1) return SPMD_ERR_INVALID_DIM;
    if (!is_pow2(B) || B < 64 || B > 1024) return SPMD_ERR_INVALID_DIM;
    auto x = arg<const int32_t*>(c.args, 0);
    auto y = arg<int32_t*>(c.args, 1);
    auto n = arg<uint32_t>(c.args, 2);
    auto ws = arg<uint32_t*>(c.args, 3);
    if (n && (!x || !y)) return SPMD_ERR_ARGS;
    if (!ws || !aligned(ws, 16)) return SPMD_ERR_WORKSPACE;
    const uint64_t per = ((uint64_t)n + (uint64_t)c.grid.x * B - 1) / ((uint64_t)c.grid.x * B);
    const uint32_t I = next_pow2(per ? (uint32_t)per : 1u);
    if (I > 32) return SPMD_ERR_INVALID_DIM;
    if (n == 0) return SPMD_OK;
    const bool vec = aligned(x, 16) && aligned(y, 16);
    dim3 g(c.grid.x);
    uint32_t* err = c.dev->err_word;
    switch (B) {
    case 64: launch_b<64>(I, g, c.dyn_shmem, c.stream, x, y, n, ws, err, vec); break;
    case 128: launch_b<128>(I, g, c.dyn_shmem, c.stream, x, y, n, ws, err, vec); break;
    case 256: launch_b<256>(I, g, c.dyn_shmem, c.stream, x, y, n, ws, err, vec); break;
    case 512: launch_b<512>(I, g, c.dyn_shmem, c.stream, x, y, n, ws, err, vec); break;
    case 1024: launch_b<1024>(I, g, c.dyn_shmem, c.stream, x, y, n, ws, err, vec); break;
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SPMD_OK : hip_fail(e);
}

}  // namespace spmd
