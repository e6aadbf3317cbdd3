// k_hist.hip -- HIST256_U32 kernels and launcher.  The launch enqueues a
// clear of the 256 output bins (a fill kernel, so the pair can be captured
// into a graph) and then the counting grid.
#include "cls_hist.hpp"

namespace spmd {

__global__ __launch_bounds__(256) void hist_clear_kernel(uint32_t* hist) { hist[threadIdx.x] = 0u; }

template <int B>
__global__ __launch_bounds__(B) void hist256_kernel(const uint32_t* __restrict__ keys, uint32_t* hist, uint32_t n,
                                                     uint32_t seg, bool vec) {
    __shared__ HistLds<HIST_COPIES> L;
    const uint64_t lo = (uint64_t)blockIdx.x * seg;
    const uint64_t hi = lo + seg < (uint64_t)n ? lo + seg : (uint64_t)n;
    hist_block<B, HIST_COPIES>(keys, hist, lo, hi, vec, L);
}

int launch_hist256_u32(const LaunchCtx& c) {
    const uint32_t B = c.block.x;
    if (c.block.y != 1 || c.block.z != 1 || c.grid.y != 1 || c.grid.z != 1) return SPMD_ERR_INVALID_DIM;
    if (!is_pow2(B) || B < 64 || B > 1024) return SPMD_ERR_INVALID_DIM;
    auto keys = arg<const uint32_t*>(c.args, 0);
    auto hist = arg<uint32_t*>(c.args, 1);
    auto n = arg<uint32_t>(c.args, 2);
    if ((!keys && n) || !hist) return SPMD_ERR_ARGS;
    const uint32_t G = c.grid.x;
    const uint64_t seg64 = segment_len(n, G);
    if (seg64 > 0xFFFFFFFFull) return SPMD_ERR_INVALID_DIM;
    const uint32_t seg = (uint32_t)seg64;
    const bool vec = aligned(keys, 16);
    dispatch(hist_clear_kernel, dim3(1), dim3(256), 0, c.stream, hist);
    if (n) {
        dim3 g(G), b(B);
        switch (B) {
        case 64: dispatch(hist256_kernel<64>, g, b, c.dyn_shmem, c.stream, keys, hist, n, seg, vec); break;
        case 128: dispatch(hist256_kernel<128>, g, b, c.dyn_shmem, c.stream, keys, hist, n, seg, vec); break;
        case 256: dispatch(hist256_kernel<256>, g, b, c.dyn_shmem, c.stream, keys, hist, n, seg, vec); break;
        case 512: dispatch(hist256_kernel<512>, g, b, c.dyn_shmem, c.stream, keys, hist, n, seg, vec); break;
        case 1024: dispatch(hist256_kernel<1024>, g, b, c.dyn_shmem, c.stream, keys, hist, n, seg, vec); break;
        }
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SPMD_OK : hip_fail(e);
}

}  // namespace spmd
