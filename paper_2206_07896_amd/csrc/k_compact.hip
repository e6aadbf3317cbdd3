// k_compact.hip -- COMPACT_I32 kernel and launcher.
//
// Workspace as for SCAN_I32 (zero-filled once): a 64-bit ticket word
// (epoch << 32 | count) alone on its cache line, then from byte 256 one u64
// status word per tile.  As for the scan, the kernel is persistent:
// min(G, resident) blocks take tiles from the ticket in order, so every
// look-back wait is for a tile a running block holds; a block draws its
// next tile once its current tile is staged (no workgroup launch between
// tiles), and the launch's last draw (G + blocks - 1) re-arms the ticket
// and advances the epoch.  A tile's count is published before the block
// waits for anything (its first tile) or once the previous tile's
// look-back has ended (every later tile); that look-back waits only for
// smaller tiles, so by induction over the tile index every wait ends.
#include <algorithm>

#include "cls_compact.hpp"

namespace spmd {

constexpr size_t COMPACT_WS_HEADER = 256;

__device__ __forceinline__ uint32_t compact_draw(uint64_t* ticket, uint32_t ntiles, uint32_t* tag) {
    const uint64_t tk = atomic_add_dev64(ticket, 1ull);
    const uint32_t cnt = (uint32_t)tk, epoch = (uint32_t)(tk >> 32);
    if (cnt == ntiles + gridDim.x - 1u)  // the launch's last draw
        __hip_atomic_store(ticket, (uint64_t)(epoch + 1u) << 32, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *tag = epoch;
    return cnt;
}

template <int B, int I>
__global__ __launch_bounds__(B) void compact_i32_kernel(const int32_t* __restrict__ x, int32_t* __restrict__ y,
                                                         uint32_t* count, uint32_t n, int32_t t, uint32_t ntiles,
                                                         uint32_t* ws, uint32_t* err, bool vec) {
    __shared__ CompactLds<B, I> L;
    __shared__ uint32_t s_next, s_tag;
    uint64_t* ticket = reinterpret_cast<uint64_t*>(ws);
    uint64_t* status = reinterpret_cast<uint64_t*>(reinterpret_cast<uint8_t*>(ws) + COMPACT_WS_HEADER);
    const uint32_t tid = threadIdx.x;
    if (tid == 0) s_next = compact_draw(ticket, ntiles, &s_tag);
    __syncthreads();
    const uint32_t tag = s_tag;
    uint32_t t0 = s_next;  // block-uniform
    if (t0 >= ntiles) return;
    CompactFront<B, I> F;
    uint32_t agg0, wpre;
    compact_issue<B, I>(x, n, t0, vec, F);
    compact_count<B, I>(x, n, t, t0, F, L);
    __syncthreads();
    compact_sums<B, I>(L, agg0, wpre);
    if (tid == 0) scan_publish_agg(status, t0, agg0, tag);
    compact_stage<B, I>(x, n, t, t0, wpre, F, L);
    if (tid == 0) {
        uint32_t unused;
        s_next = compact_draw(ticket, ntiles, &unused);
    }
    __syncthreads();  // t0 staged, s_next visible
    // Tile t0 is staged and its count published.  The next tile t1 is drawn
    // already: its loads are issued before t0's look-back, and its count is
    // published before t0's copy-out, so no successor waits on t1 for the
    // length of t0's copy-out.
    for (;;) {
        const uint32_t t1 = s_next;
        const bool has1 = t1 < ntiles;
        if (has1) compact_issue<B, I>(x, n, t1, vec, F);
        if (tid < 64) {
            const uint32_t excl = scan_lookback(status, t0, agg0, tag, err, true);
            if (tid == 0) {
                L.excl = excl;
                if (t0 == ntiles - 1) *count = excl + agg0;
            }
        }
        if (has1) compact_count<B, I>(x, n, t, t1, F, L);
        __syncthreads();  // L.excl, and t1's warp counts
        uint32_t agg1 = 0;
        if (has1) {
            compact_sums<B, I>(L, agg1, wpre);
            if (tid == 0) scan_publish_agg(status, t1, agg1, tag);
        }
        int32_t* yo = y + L.excl;
        for (uint32_t i = tid; i < agg0; i += B) yo[i] = (int32_t)L.stage[i];
        __syncthreads();  // the stage, L.excl and L.warp are free again
        if (!has1) break;
        compact_stage<B, I>(x, n, t, t1, wpre, F, L);
        if (tid == 0) {
            uint32_t unused;
            s_next = compact_draw(ticket, ntiles, &unused);
        }
        __syncthreads();
        t0 = t1;
        agg0 = agg1;
    }
}

size_t ws_compact_i32(spmd_dim3 grid, spmd_dim3, uint64_t) { return COMPACT_WS_HEADER + 8ull * grid.x; }

template <int B, int I>
static void launch_bi(uint32_t G, size_t dyn, hipStream_t s, const int32_t* x, int32_t* y, uint32_t* cnt,
                      uint32_t n, int32_t t, uint32_t* ws, uint32_t* err, bool vec, int num_cus) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, compact_i32_kernel<B, I>, B, dyn) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    const uint32_t P = (uint32_t)std::min<uint64_t>(G, (uint64_t)per_cu * (uint64_t)num_cus);
    dispatch((compact_i32_kernel<B, I>), dim3(P), dim3(B), dyn, s, x, y, cnt, n, t, G, ws, err, vec);
}

template <int B>
static void launch_b(uint32_t I, uint32_t G, size_t dyn, hipStream_t s, const int32_t* x, int32_t* y, uint32_t* cnt,
                     uint32_t n, int32_t t, uint32_t* ws, uint32_t* err, bool vec, int num_cus) {
    switch (I) {
    case 1: launch_bi<B, 1>(G, dyn, s, x, y, cnt, n, t, ws, err, vec, num_cus); break;
    case 2: launch_bi<B, 2>(G, dyn, s, x, y, cnt, n, t, ws, err, vec, num_cus); break;
    case 4: launch_bi<B, 4>(G, dyn, s, x, y, cnt, n, t, ws, err, vec, num_cus); break;
    case 8: launch_bi<B, 8>(G, dyn, s, x, y, cnt, n, t, ws, err, vec, num_cus); break;
    case 16: launch_bi<B, 16>(G, dyn, s, x, y, cnt, n, t, ws, err, vec, num_cus); break;
    case 32: launch_bi<B, 32>(G, dyn, s, x, y, cnt, n, t, ws, err, vec, num_cus); break;
    case 64:
        if constexpr (B <= 512) launch_bi<B, 64>(G, dyn, s, x, y, cnt, n, t, ws, err, vec, num_cus);
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
    if (overlap(x, 4ull * n, y, 4ull * n) || overlap(x, 4ull * n, cnt, 4)) return SPMD_ERR_ARGS;
    if (!ws || !aligned(ws, 16)) return SPMD_ERR_WORKSPACE;
    const uint64_t per = ((uint64_t)n + (uint64_t)c.grid.x * B - 1) / ((uint64_t)c.grid.x * B);
    const uint32_t I = next_pow2(per ? (uint32_t)per : 1u);
    if (I > 64 || (I == 64 && B > 512)) return SPMD_ERR_INVALID_DIM;
    const bool vec = aligned(x, 16);
    const uint32_t G = c.grid.x;
    uint32_t* err = c.dev->err_word;
    const int cus = c.dev->num_cus;
    switch (B) {
    case 64: launch_b<64>(I, G, c.dyn_shmem, c.stream, x, y, cnt, n, t, ws, err, vec, cus); break;
    case 128: launch_b<128>(I, G, c.dyn_shmem, c.stream, x, y, cnt, n, t, ws, err, vec, cus); break;
    case 256: launch_b<256>(I, G, c.dyn_shmem, c.stream, x, y, cnt, n, t, ws, err, vec, cus); break;
    case 512: launch_b<512>(I, G, c.dyn_shmem, c.stream, x, y, cnt, n, t, ws, err, vec, cus); break;
    case 1024: launch_b<1024>(I, G, c.dyn_shmem, c.stream, x, y, cnt, n, t, ws, err, vec, cus); break;
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SPMD_OK : hip_fail(e);
}

}  // namespace spmd
