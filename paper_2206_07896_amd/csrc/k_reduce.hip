// k_reduce.hip -- REDUCE_I32 kernel and launcher.
//
// Workspace: the two-level completion ticket and the launch epoch
// (REDUCE_CTL_BYTES, counters on separate cache lines), then one u64 status
// word per block (per workgroup in the persistent form, which needs fewer),
// tagged with the epoch: the finishing block re-arms the ticket and
// advances the epoch, so the next launch needs no clearing.
#include "cls_reduce.hpp"
#include "common.hpp"

namespace spmd {

constexpr size_t REDUCE_WS_HEADER = REDUCE_CTL_BYTES;

template <int B>
__global__ __launch_bounds__(B) void reduce_i32_kernel(const int32_t* __restrict__ x, int32_t* partials,
                                                        int32_t* out, uint32_t n, uint32_t seg, uint32_t* ws,
                                                        uint32_t* err, bool vec) {
    __shared__ ReduceLds<B> L;
    uint64_t* status = reinterpret_cast<uint64_t*>(reinterpret_cast<uint8_t*>(ws) + REDUCE_WS_HEADER);
    reduce_block<B>(x, partials, out, n, seg, gridDim.x, blockIdx.x, ws, status, err, vec, L);
}

// The persistent form: workgroup w runs logical blocks [K w, K w + K).
template <int B, int K>
__global__ __launch_bounds__(B) void reduce_i32_pkernel(const int32_t* __restrict__ x, int32_t* partials,
                                                         int32_t* out, uint32_t n, uint32_t seg, uint32_t G,
                                                         uint32_t* ws, uint32_t* err, bool vec) {
    __shared__ ReduceLds<B> L;
    __shared__ uint32_t wsum[K][B / 64];
    uint64_t* status = reinterpret_cast<uint64_t*>(reinterpret_cast<uint8_t*>(ws) + REDUCE_WS_HEADER);
    reduce_blocks<B, K>(x, partials, out, n, seg, G, gridDim.x, blockIdx.x, ws, status, err, vec, L, wsum);
}

size_t ws_reduce_i32(spmd_dim3 grid, spmd_dim3, uint64_t) { return REDUCE_WS_HEADER + 8ull * grid.x; }

// Logical blocks per workgroup: the largest K in {1, 2, 4, 8} that still
// leaves at least one workgroup per resident slot (2 for the 2^20 x 4096 x
// 256 configuration: 2048 workgroups of 256 threads fill the device).  At
// K = 1 the one-block-per-workgroup kernel runs.
template <int B>
static uint32_t reduce_blocks_per_wg(uint32_t G, int num_cus) {
    static const int per_cu = [] {  // one query per block size (one GPU architecture)
        int v = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, reduce_i32_pkernel<B, 2>, B, 0) != hipSuccess) v = 0;
        return v;
    }();
    if (per_cu < 1) return 1;
    const uint64_t slots = (uint64_t)per_cu * (uint64_t)num_cus;
    uint32_t K = 1;
    while (K < 8 && (uint64_t)G >= 2ull * K * slots) K *= 2;
    return K;
}

template <int B>
static void launch_reduce_b(uint32_t G, size_t dyn, hipStream_t s, const int32_t* x, int32_t* partials,
                            int32_t* out, uint32_t n, uint32_t seg, uint32_t* ws, uint32_t* err, bool vec,
                            int num_cus) {
    const uint32_t K = reduce_blocks_per_wg<B>(G, num_cus);
    const dim3 b(B);
    switch (K) {
    case 1: dispatch(reduce_i32_kernel<B>, dim3(G), b, dyn, s, x, partials, out, n, seg, ws, err, vec); break;
    case 2: dispatch((reduce_i32_pkernel<B, 2>), dim3((G + 1) / 2), b, dyn, s, x, partials, out, n, seg, G, ws, err, vec); break;
    case 4: dispatch((reduce_i32_pkernel<B, 4>), dim3((G + 3) / 4), b, dyn, s, x, partials, out, n, seg, G, ws, err, vec); break;
    default: dispatch((reduce_i32_pkernel<B, 8>), dim3((G + 7) / 8), b, dyn, s, x, partials, out, n, seg, G, ws, err, vec); break;
    }
}

int launch_reduce_i32(const LaunchCtx& c) {
    const uint32_t B = c.block.x;
    if (c.block.y != 1 || c.block.z != 1 || c.grid.y != 1 || c.grid.z != 1) return SPMD_ERR_INVALID_DIM;
    if (!is_pow2(B) || B < 64 || B > 1024) return SPMD_ERR_INVALID_DIM;
    auto x = arg<const int32_t*>(c.args, 0);
    auto partials = arg<int32_t*>(c.args, 1);
    auto out = arg<int32_t*>(c.args, 2);
    auto n = arg<uint32_t>(c.args, 3);
    auto ws = arg<uint32_t*>(c.args, 4);
    if ((!x && n) || !partials || !out) return SPMD_ERR_ARGS;
    if (!ws || !aligned(ws, 16)) return SPMD_ERR_WORKSPACE;
    const uint32_t G = c.grid.x;
    const uint64_t seg64 = segment_len(n, G);
    if (seg64 > 0xFFFFFFFFull) return SPMD_ERR_INVALID_DIM;
    const uint32_t seg = (uint32_t)seg64;
    const bool vec = aligned(x, 16);
    uint32_t* err = c.dev->err_word;
    const int cus = c.dev->num_cus;
    switch (B) {
    case 64: launch_reduce_b<64>(G, c.dyn_shmem, c.stream, x, partials, out, n, seg, ws, err, vec, cus); break;
    case 128: launch_reduce_b<128>(G, c.dyn_shmem, c.stream, x, partials, out, n, seg, ws, err, vec, cus); break;
    case 256: launch_reduce_b<256>(G, c.dyn_shmem, c.stream, x, partials, out, n, seg, ws, err, vec, cus); break;
    case 512: launch_reduce_b<512>(G, c.dyn_shmem, c.stream, x, partials, out, n, seg, ws, err, vec, cus); break;
    case 1024: launch_reduce_b<1024>(G, c.dyn_shmem, c.stream, x, partials, out, n, seg, ws, err, vec, cus); break;
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SPMD_OK : hip_fail(e);
}

}  // namespace spmd
