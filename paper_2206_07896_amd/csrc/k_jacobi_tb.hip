// k_jacobi_tb.hip -- JACOBI5T_F32 kernel and launcher: S fused sweeps.
#include "cls_jacobi_tb.hpp"

namespace spmd {

template <int H>
__global__ __launch_bounds__(JT_THREADS) void jacobi5_tb_kernel(const float* __restrict__ u, float* __restrict__ v,
                                                                uint32_t nx, uint32_t ny, uint32_t sweeps) {
    __shared__ JacobiTbLds L;
    const uint32_t nt = gridDim.x * gridDim.y;
    const uint32_t tile = xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, nt);
    jacobi_tb_block<H>(u, v, nx, ny, sweeps, tile % gridDim.x, tile / gridDim.x, L);
}

int launch_jacobi5t_f32(const LaunchCtx& c) {
    if (c.block.x != (uint32_t)JT_THREADS || c.block.y != 1 || c.block.z != 1 || c.grid.z != 1)
        return SPMD_ERR_INVALID_DIM;
    auto u = arg<const float*>(c.args, 0);
    auto v = arg<float*>(c.args, 1);
    auto nx = arg<uint32_t>(c.args, 2);
    auto ny = arg<uint32_t>(c.args, 3);
    auto sweeps = arg<uint32_t>(c.args, 4);
    if (!u || !v || nx == 0 || ny == 0 || sweeps == 0 || sweeps > 8) return SPMD_ERR_ARGS;
    if (nx % 4u || !aligned(u, 16) || !aligned(v, 16)) return SPMD_ERR_ARGS;
    const uint64_t bytes = 4ull * nx * ny;
    const uintptr_t a = (uintptr_t)u, b = (uintptr_t)v;
    if (a < b + bytes && b < a + bytes) return SPMD_ERR_ARGS;  // u and v overlap
    const int halo = sweeps <= 4 ? 4 : 8;
    if ((uint64_t)c.grid.x * jt_width(halo) < nx || (uint64_t)c.grid.y * JT_H < ny) return SPMD_ERR_INVALID_DIM;
    const dim3 g(c.grid.x, c.grid.y), bl(JT_THREADS);
    if (sweeps <= 4)
        dispatch((jacobi5_tb_kernel<4>), g, bl, c.dyn_shmem, c.stream, u, v, nx, ny, sweeps);
    else
        dispatch((jacobi5_tb_kernel<8>), g, bl, c.dyn_shmem, c.stream, u, v, nx, ny, sweeps);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SPMD_OK : hip_fail(e);
}

}  // namespace spmd
