// k_scan.hip -- SCAN_I32 kernels and launcher.
//
// Workspace (zero-filled once): a 64-bit ticket word (epoch << 32 | count)
// alone on its cache line, then from byte 256 one u64 status word per
// tile.  A block takes its tile index from the ticket when it starts, so
// tiles start in index order and a tile only waits for tiles that started
// before it: every wait ends.  The ticket's high half is the launch's epoch,
// the tag of its status words; the block that draws count G-1 -- every
// block of the launch has drawn by then -- re-arms the count and advances
// the epoch.  One atomic per tile, nothing to clear between launches.
#include "cls_scan.hpp"

namespace spmd {

constexpr size_t SCAN_WS_HEADER = 256;

template <int B, int I>
__global__ __launch_bounds__(B) void scan_i32_kernel(const int32_t* __restrict__ x, int32_t* __restrict__ y,
                                                      uint32_t n, uint32_t* ws, uint32_t* err, bool vec) {
    __shared__ ScanLds<B, I> L;
    __shared__ uint32_t s_tile, s_tag;
    uint64_t* ticket = reinterpret_cast<uint64_t*>(ws);
    uint64_t* status = reinterpret_cast<uint64_t*>(reinterpret_cast<uint8_t*>(ws) + SCAN_WS_HEADER);
    if (threadIdx.x == 0) {
        const uint64_t tk = atomic_add_dev64(ticket, 1ull);
        const uint32_t count = (uint32_t)tk, epoch = (uint32_t)(tk >> 32);
        if (count == gridDim.x - 1u)
            __hip_atomic_store(ticket, (uint64_t)(epoch + 1u) << 32, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_tile = count;
        s_tag = epoch;
    }
    __syncthreads();
    scan_tile<B, I>(x, y, n, s_tile, status, s_tag, err, vec, L);
}

size_t ws_scan_i32(spmd_dim3 grid, spmd_dim3, uint64_t) { return SCAN_WS_HEADER + 8ull * grid.x; }

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
    case 64:
        if constexpr (B <= 512) hipLaunchKernelGGL((scan_i32_kernel<B, 64>), g, b, dyn, s, x, y, n, ws, err, vec);
        break;
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
    if (I > 64 || (I == 64 && B > 512)) return SPMD_ERR_INVALID_DIM;
    if (n == 0) return SPMD_OK;
    const bool vec = aligned(x, 16) && aligned(y, 16);
    const uint32_t G = c.grid.x;
    dim3 g(G);
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
