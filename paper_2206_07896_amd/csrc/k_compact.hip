// k_compact.hip -- COMPACT_I32 kernel and launcher.
//
// Workspace as for SCAN_I32 (zero-filled once): a 64-bit ticket word
// (epoch << 32 | count) alone on its cache line, then from byte 256 one u64
// status word per tile.  Tiles take their index from the ticket in start
// order, so every look-back wait is for a tile that has started; the block
// that draws the last count re-arms the ticket and advances the epoch.
#include "cls_compact.hpp"

namespace spmd {

constexpr size_t COMPACT_WS_HEADER = 256;

template <int B, int I>
__global__ __launch_bounds__(B) void compact_i32_kernel(const int32_t* __restrict__ x, int32_t* __restrict__ y,
                                                         uint32_t* count, uint32_t n, int32_t t, uint32_t* ws,
                                                         uint32_t* err, bool vec) {
    __shared__ CompactLds<B, I> L;
    __shared__ uint32_t s_tile, s_tag;
    uint64_t* ticket = reinterpret_cast<uint64_t*>(ws);
    uint64_t* status = reinterpret_cast<uint64_t*>(reinterpret_cast<uint8_t*>(ws) + COMPACT_WS_HEADER);
    if (threadIdx.x == 0) {
        const uint64_t tk = atomic_add_dev64(ticket, 1ull);
        const uint32_t cnt = (uint32_t)tk, epoch = (uint32_t)(tk >> 32);
        if (cnt == gridDim.x - 1u)
            __hip_atomic_store(ticket, (uint64_t)(epoch + 1u) << 32, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_tile = cnt;
        s_tag = epoch;
    }
    __syncthreads();
    compact_tile<B, I>(x, y, count, n, t, s_tile, gridDim.x, status, s_tag, err, vec, L);
}

size_t ws_compact_i32(spmd_dim3 grid, spmd_dim3, uint64_t) { return COMPACT_WS_HEADER + 8ull * grid.x; }

template <int B>
static void launch_b(uint32_t I, dim3 g, size_t dyn, hipStream_t s, const int32_t* x, int32_t* y, uint32_t* cnt,
                     uint32_t n, int32_t t, uint32_t* ws, uint32_t* err, bool vec) {
    dim3 b(B);
    switch (I) {
    case 1: hipLaunchKernelGGL((compact_i32_kernel<B, 1>), g, b, dyn, s, x, y, cnt, n, t, ws, err, vec); break;
    case 2: hipLaunchKernelGGL((compact_i32_kernel<B, 2>), g, b, dyn, s, x, y, cnt, n, t, ws, err, vec); break;
    case 4: hipLaunchKernelGGL((compact_i32_kernel<B, 4>), g, b, dyn, s, x, y, cnt, n, t, ws, err, vec); break;
    case 8: hipLaunchKernelGGL((compact_i32_kernel<B, 8>), g, b, dyn, s, x, y, cnt, n, t, ws, err, vec); break;
    case 16: hipLaunchKernelGGL((compact_i32_kernel<B, 16>), g, b, dyn, s, x, y, cnt, n, t, ws, err, vec); break;
    case 32: hipLaunchKernelGGL((compact_i32_kernel<B, 32>), g, b, dyn, s, x, y, cnt, n, t, ws, err, vec); break;
    case 64:
        if constexpr (B <= 512) hipLaunchKernelGGL((compact_i32_kernel<B, 64>), g, b, dyn, s, x, y, cnt, n, t, ws, err, vec);
        break;
    }
}

int launch_compact_i32(const LaunchCtx& c) {
    const uint32_t B = c.block.x;
    if (c.block.y != 1 || c.block.z != 1 || c.grid.y != 1 || c.grid.z != 1) return SPMD_ERR_INVALID_DIM;
    if (!is_pow2(B) || B < 64 || B > 1024) return SPMD_ERR_INVALID_DIM;
    auto x = arg<const int32_t*>(c.args, 0);
    auto y = arg<int32_t*>(c.args, 1);
    auto cnt = arg<uint32_t*>(c.args, 2);
    auto n = arg<uint32_t>(c.args, 3);
    auto t = (int32_t)arg<uint32_t>(c.args, 4);
    auto ws = arg<uint32_t*>(c.args, 5);
    if (!cnt || (n && (!x || !y))) return SPMD_ERR_ARGS;
    if (!ws || !aligned(ws, 16)) return SPMD_ERR_WORKSPACE;
    const uint64_t per = ((uint64_t)n + (uint64_t)c.grid.x * B - 1) / ((uint64_t)c.grid.x * B);
    const uint32_t I = next_pow2(per ? (uint32_t)per : 1u);
    if (I > 64 || (I == 64 && B > 512)) return SPMD_ERR_INVALID_DIM;
    const bool vec = aligned(x, 16);
    dim3 g(c.grid.x);
    uint32_t* err = c.dev->err_word;
    switch (B) {
    case 64: launch_b<64>(I, g, c.dyn_shmem, c.stream, x, y, cnt, n, t, ws, err, vec); break;
    case 128: launch_b<128>(I, g, c.dyn_shmem, c.stream, x, y, cnt, n, t, ws, err, vec); break;
    case 256: launch_b<256>(I, g, c.dyn_shmem, c.stream, x, y, cnt, n, t, ws, err, vec); break;
    case 512: launch_b<512>(I, g, c.dyn_shmem, c.stream, x, y, cnt, n, t, ws, err, vec); break;
    case 1024: launch_b<1024>(I, g, c.dyn_shmem, c.stream, x, y, cnt, n, t, ws, err, vec); break;
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SPMD_OK : hip_fail(e);
}

}  // namespace spmd
