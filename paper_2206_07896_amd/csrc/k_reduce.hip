// k_reduce.hip -- REDUCE_I32 kernel and launcher.
//
// Workspace: the two-level completion ticket and the launch epoch
// (REDUCE_CTL_BYTES, counters on separate cache lines), then one u64 status
// word per block, tagged with the epoch: the finishing block re-arms the
// ticket and advances the epoch, so the next launch needs no clearing.
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

size_t ws_reduce_i32(spmd_dim3 grid, spmd_dim3, uint64_t) { return REDUCE_WS_HEADER + 8ull * grid.x; }

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
    dim3 g(G), b(B);
    switch (B) {
    case 64: hipLaunchKernelGGL(reduce_i32_kernel<64>, g, b, c.dyn_shmem, c.stream, x, partials, out, n, seg, ws, err, vec); break;
    case 128: hipLaunchKernelGGL(reduce_i32_kernel<128>, g, b, c.dyn_shmem, c.stream, x, partials, out, n, seg, ws, err, vec); break;
    case 256: hipLaunchKernelGGL(reduce_i32_kernel<256>, g, b, c.dyn_shmem, c.stream, x, partials, out, n, seg, ws, err, vec); break;
    case 512: hipLaunchKernelGGL(reduce_i32_kernel<512>, g, b, c.dyn_shmem, c.stream, x, partials, out, n, seg, ws, err, vec); break;
    case 1024: hipLaunchKernelGGL(reduce_i32_kernel<1024>, g, b, c.dyn_shmem, c.stream, x, partials, out, n, seg, ws, err, vec); break;
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SPMD_OK : hip_fail(e);
}

}  // namespace spmd
