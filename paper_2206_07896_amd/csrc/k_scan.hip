// k_scan.hip -- SCAN_I32 kernels and launcher.
//
// Workspace (zero-filled once): a 64-bit ticket word (epoch << 32 | count)
// alone on its cache line, then from byte 256 one u64 status word per
// tile.  Tiles are handed out by the ticket, so they start in index order
// and a tile only waits for tiles that a running block already holds: every
// wait ends.  The ticket's high half is the launch's epoch, the tag of its
// status words.
//
// The kernel is persistent: P = min(G, resident blocks) blocks loop over the
// G tiles.  A block draws its next ticket as soon as its current tile has
// published its inclusive prefix (no tile can wait on it any more), so the
// draw's round trip overlaps the tile's stores and the next tile starts
// without a workgroup launch.  A draw >= G ends the block; each block makes
// exactly one such draw, so the launch makes G + P draws in all, and the
// block that makes the last one re-arms the count and advances the epoch.
// One atomic per tile plus one per block, nothing to clear between
// launches.
#include <algorithm>

#include "cls_scan.hpp"

namespace spmd {

constexpr size_t SCAN_WS_HEADER = 256;

// Draw a ticket (thread 0): the tile index, or a value >= ntiles to stop.
__device__ __forceinline__ uint32_t scan_draw(uint64_t* ticket, uint32_t ntiles, uint32_t* tag) {
    const uint64_t tk = atomic_add_dev64(ticket, 1ull);
    const uint32_t count = (uint32_t)tk, epoch = (uint32_t)(tk >> 32);
    if (count == ntiles + gridDim.x - 1u)  // the launch's last draw
        __hip_atomic_store(ticket, (uint64_t)(epoch + 1u) << 32, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *tag = epoch;
    return count;
}

template <int B, int I>
__global__ __launch_bounds__(B) void scan_i32_kernel(const int32_t* __restrict__ x, int32_t* __restrict__ y,
                                                      uint32_t n, uint32_t ntiles, uint32_t* ws, uint32_t* err,
                                                      bool vec) {
    __shared__ ScanLds<B, I> L;
    __shared__ uint32_t s_tile, s_next, s_tag;
    uint64_t* ticket = reinterpret_cast<uint64_t*>(ws);
    uint64_t* status = reinterpret_cast<uint64_t*>(reinterpret_cast<uint8_t*>(ws) + SCAN_WS_HEADER);
    if (threadIdx.x == 0) s_tile = scan_draw(ticket, ntiles, &s_tag);
    __syncthreads();
    uint32_t tile = s_tile;
    const uint32_t tag = s_tag;  // every draw of a launch carries its epoch
    while (tile < ntiles) {
        auto draw_next = [&]() {
            uint32_t unused;
            s_next = scan_draw(ticket, ntiles, &unused);
        };
        scan_tile<B, I>(x, y, n, tile, status, tag, err, vec, L, draw_next);
        // No barrier here: s_next is written before the tile's second
        // barrier, and thread 0 writes it, L.excl and L.warp again only after
        // the next tile's first barrier, which every thread reaches after
        // its last read of them.
        tile = s_next;
    }
}

size_t ws_scan_i32(spmd_dim3 grid, spmd_dim3, uint64_t) { return SCAN_WS_HEADER + 8ull * grid.x; }

// Persistent grid for G tiles: at most the blocks that are resident at once.
template <int B, int I>
static void launch_bi(uint32_t G, size_t dyn, hipStream_t s, const int32_t* x, int32_t* y, uint32_t n,
                      uint32_t* ws, uint32_t* err, bool vec, int num_cus) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, scan_i32_kernel<B, I>, B, dyn) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    const uint32_t P = (uint32_t)std::min<uint64_t>(G, (uint64_t)per_cu * (uint64_t)num_cus);
    dispatch((scan_i32_kernel<B, I>), dim3(P), dim3(B), dyn, s, x, y, n, G, ws, err, vec);
}

template <int B>
static void launch_b(uint32_t I, uint32_t G, size_t dyn, hipStream_t s, const int32_t* x, int32_t* y, uint32_t n,
                     uint32_t* ws, uint32_t* err, bool vec, int num_cus) {
    switch (I) {
    case 1: launch_bi<B, 1>(G, dyn, s, x, y, n, ws, err, vec, num_cus); break;
    case 2: launch_bi<B, 2>(G, dyn, s, x, y, n, ws, err, vec, num_cus); break;
    case 4: launch_bi<B, 4>(G, dyn, s, x, y, n, ws, err, vec, num_cus); break;
    case 8: launch_bi<B, 8>(G, dyn, s, x, y, n, ws, err, vec, num_cus); break;
    case 16: launch_bi<B, 16>(G, dyn, s, x, y, n, ws, err, vec, num_cus); break;
    case 32: launch_bi<B, 32>(G, dyn, s, x, y, n, ws, err, vec, num_cus); break;
    case 64:
        if constexpr (B <= 512) launch_bi<B, 64>(G, dyn, s, x, y, n, ws, err, vec, num_cus);
        break;
    case 128:
        if constexpr (B <= 512) launch_bi<B, 128>(G, dyn, s, x, y, n, ws, err, vec, num_cus);
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
    if (overlap(x, 4ull * n, y, 4ull * n)) return SPMD_ERR_ARGS;
    if (!ws || !aligned(ws, 16)) return SPMD_ERR_WORKSPACE;
    const uint64_t per = ((uint64_t)n + (uint64_t)c.grid.x * B - 1) / ((uint64_t)c.grid.x * B);
    const uint32_t I = next_pow2(per ? (uint32_t)per : 1u);
    if (I > 128 || (I >= 64 && B > 512)) return SPMD_ERR_INVALID_DIM;  // 1024 x 64 would spill
    if (n == 0) return SPMD_OK;
    const bool vec = aligned(x, 16) && aligned(y, 16);
    const uint32_t G = c.grid.x;
    uint32_t* err = c.dev->err_word;
    const int cus = c.dev->num_cus;
    switch (B) {
    case 64: launch_b<64>(I, G, c.dyn_shmem, c.stream, x, y, n, ws, err, vec, cus); break;
    case 128: launch_b<128>(I, G, c.dyn_shmem, c.stream, x, y, n, ws, err, vec, cus); break;
    case 256: launch_b<256>(I, G, c.dyn_shmem, c.stream, x, y, n, ws, err, vec, cus); break;
    case 512: launch_b<512>(I, G, c.dyn_shmem, c.stream, x, y, n, ws, err, vec, cus); break;
    case 1024: launch_b<1024>(I, G, c.dyn_shmem, c.stream, x, y, n, ws, err, vec, cus); break;
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SPMD_OK : hip_fail(e);
}

}  // namespace spmd
