// k_gemm.hip -- GEMM_F32 kernel and launcher.
#include "cls_gemm.hpp"

namespace spmd {

template <int T>
__global__ __launch_bounds__(256) void gemm_f32_kernel(const float* __restrict__ A, const float* __restrict__ B,
                                                        float* __restrict__ C, uint32_t M, uint32_t N, uint32_t K,
                                                        bool vecA, bool vecB) {
    __shared__ GemmLds<T> L;
    gemm_block<T>(A, B, C, M, N, K, blockIdx.x, blockIdx.y, vecA, vecB, L);
}

// Direct-to-LDS form: NS slices in flight (4 at tiles 64 and 128; 3 at
// tile 256, whose stages are twice as large).
template <int T, int NS>
__global__ __launch_bounds__(256) void gemm_f32_dma_kernel(const float* __restrict__ A, const float* __restrict__ B,
                                                            float* __restrict__ C, uint32_t M, uint32_t N, uint32_t K) {
    constexpr int SZ = 2 * T * GEMM_DMA_KT;
    __shared__ __attribute__((aligned(16))) float S0[SZ];
    __shared__ __attribute__((aligned(16))) float S1[SZ];
    __shared__ __attribute__((aligned(16))) float S2[NS > 2 ? SZ : 4];
    __shared__ __attribute__((aligned(16))) float S3[NS > 3 ? SZ : 4];
    gemm_block_dma<T, NS>(A, B, C, M, N, K, blockIdx.x, blockIdx.y, S0, S1, S2, S3);
}

int launch_gemm_f32(const LaunchCtx& c) {
    if (c.block.x != 256 || c.block.y != 1 || c.block.z != 1 || c.grid.z != 1) return SPMD_ERR_INVALID_DIM;
    auto A = arg<const float*>(c.args, 0);
    auto B = arg<const float*>(c.args, 1);
    auto C = arg<float*>(c.args, 2);
    auto M = arg<uint32_t>(c.args, 3);
    auto N = arg<uint32_t>(c.args, 4);
    auto K = arg<uint32_t>(c.args, 5);
    if (!A || !B || !C || M == 0 || N == 0 || K == 0) return SPMD_ERR_ARGS;
    int T = 0;
    for (int t : {64, 128, 256})
        if ((uint64_t)c.grid.x * t >= N && (uint64_t)c.grid.y * t >= M) {
            T = t;
            break;
        }
    if (!T) return SPMD_ERR_INVALID_DIM;
    const bool vecA = aligned(A, 16) && (K % 4 == 0);
    const bool vecB = aligned(B, 16) && (N % 4 == 0);
    dim3 g(c.grid.x, c.grid.y), b(256);
    // The direct-to-LDS form needs 16-byte rows and 32-bit per-lane offsets.
    const bool dma = vecA && vecB && (uint64_t)T * K < (1ull << 31) && (uint64_t)GEMM_DMA_KT * N < (1ull << 31);
    if (dma) {
        if (T == 64)
            dispatch((gemm_f32_dma_kernel<64, 4>), g, b, c.dyn_shmem, c.stream, A, B, C, M, N, K);
        else if (T == 128)
            dispatch((gemm_f32_dma_kernel<128, 4>), g, b, c.dyn_shmem, c.stream, A, B, C, M, N, K);
        else
            dispatch((gemm_f32_dma_kernel<256, 3>), g, b, c.dyn_shmem, c.stream, A, B, C, M, N, K);
    } else if (T == 64)
        dispatch(gemm_f32_kernel<64>, g, b, c.dyn_shmem, c.stream, A, B, C, M, N, K, vecA, vecB);
    else if (T == 128)
        dispatch(gemm_f32_kernel<128>, g, b, c.dyn_shmem, c.stream, A, B, C, M, N, K, vecA, vecB);
    else  // 128 x 128 per wave: 256 accumulators in AGPRs, one wave per SIMD
        dispatch(gemm_f32_kernel<256>, g, b, c.dyn_shmem, c.stream, A, B, C, M, N, K, vecA, vecB);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SPMD_OK : hip_fail(e);
}

}  // namespace spmd
