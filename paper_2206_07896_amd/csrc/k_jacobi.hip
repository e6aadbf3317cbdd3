// k_jacobi.hip -- JACOBI5_F32 kernel and launcher.
#include "cls_jacobi.hpp"

namespace spmd {

template <int BX, int BY, int C>
__global__ __launch_bounds__(BX* BY) void jacobi5_kernel(const float* __restrict__ u, float* __restrict__ v,
                                                          uint32_t nx, uint32_t ny) {
    __shared__ JacobiLds<BX, BY, C> L;
    jacobi_block<BX, BY, C>(u, v, nx, ny, blockIdx.x, blockIdx.y, threadIdx.x, threadIdx.y, L);
}

template <int BY, int C>
__global__ __launch_bounds__(64 * BY) void jacobi5_v4_kernel(const float* __restrict__ u, float* __restrict__ v,
                                                             uint32_t nx, uint32_t ny) {
    __shared__ JacobiV4Lds<BY, C> L;
    const uint32_t nt = gridDim.x * gridDim.y;
    const uint32_t t = xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, nt);
    jacobi_block_v4<BY, C>(u, v, nx, ny, t % gridDim.x, t / gridDim.x, threadIdx.x, threadIdx.y, L);
}

template <int BY, int C>
__global__ __launch_bounds__(64 * BY) void jacobi5_w_kernel(const float* __restrict__ u, float* __restrict__ v,
                                                            uint32_t nx, uint32_t ny) {
    __shared__ JacobiWLds<BY, C> L;
    const uint32_t nt = gridDim.x * gridDim.y;
    const uint32_t t = xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, nt);
    jacobi_block_w<BY, C>(u, v, nx, ny, t % gridDim.x, t / gridDim.x, threadIdx.x, threadIdx.y, L);
}

template <int BX, int BY>
static void launch_c(uint32_t C, dim3 g, size_t dyn, hipStream_t s, const float* u, float* v, uint32_t nx,
                     uint32_t ny) {
    dim3 b(BX, BY);
    switch (C) {
    case 1: dispatch((jacobi5_kernel<BX, BY, 1>), g, b, dyn, s, u, v, nx, ny); break;
    case 2: dispatch((jacobi5_kernel<BX, BY, 2>), g, b, dyn, s, u, v, nx, ny); break;
    case 4: dispatch((jacobi5_kernel<BX, BY, 4>), g, b, dyn, s, u, v, nx, ny); break;
    case 8: dispatch((jacobi5_kernel<BX, BY, 8>), g, b, dyn, s, u, v, nx, ny); break;
    case 16: dispatch((jacobi5_kernel<BX, BY, 16>), g, b, dyn, s, u, v, nx, ny); break;
    }
}

int launch_jacobi5_f32(const LaunchCtx& c) {
    const uint32_t BX = c.block.x, BY = c.block.y;
    if (c.block.z != 1 || c.grid.z != 1) return SPMD_ERR_INVALID_DIM;
    auto u = arg<const float*>(c.args, 0);
    auto v = arg<float*>(c.args, 1);
    auto nx = arg<uint32_t>(c.args, 2);
    auto ny = arg<uint32_t>(c.args, 3);
    if (!u || !v || nx == 0 || ny == 0) return SPMD_ERR_ARGS;
    if ((uint64_t)c.grid.x * BX < nx) return SPMD_ERR_INVALID_DIM;
    const uint64_t rows = (uint64_t)c.grid.y * BY;
    const uint64_t per = (ny + rows - 1) / rows;
    const uint32_t C = next_pow2((uint32_t)per);
    if (C > 16) return SPMD_ERR_INVALID_DIM;
    dim3 g(c.grid.x, c.grid.y);
    const size_t d = c.dyn_shmem;
    const uint64_t brow = (uint64_t)BY * C;  // rows of one block row of the launch
    if (brow >= 4 && brow <= 64) {
        // The blocks of one block row are fetched 256 columns at a time
        // (coarse-grained fetching along x, Section IV-A) and run as one
        // workgroup of 64 x 4 threads, four columns per thread, the same
        // rows as the launch's blocks, every cell computed as in its own
        // block: 16-byte loads and stores when nx is a multiple of 4 and
        // the rows are 16-byte aligned, else four 4-byte columns 64 apart.
        const bool vec = nx % 4u == 0 && aligned(u, 16) && aligned(v, 16);
        const dim3 gv((nx + JV_W - 1) / JV_W, c.grid.y), bv(64, 4);
        hipStream_t st = c.stream;
        switch (brow) {
        case 4:
            if (vec) dispatch((jacobi5_v4_kernel<4, 1>), gv, bv, d, st, u, v, nx, ny);
            else dispatch((jacobi5_w_kernel<4, 1>), gv, bv, d, st, u, v, nx, ny);
            break;
        case 8:
            if (vec) dispatch((jacobi5_v4_kernel<4, 2>), gv, bv, d, st, u, v, nx, ny);
            else dispatch((jacobi5_w_kernel<4, 2>), gv, bv, d, st, u, v, nx, ny);
            break;
        case 16:
            if (vec) dispatch((jacobi5_v4_kernel<4, 4>), gv, bv, d, st, u, v, nx, ny);
            else dispatch((jacobi5_w_kernel<4, 4>), gv, bv, d, st, u, v, nx, ny);
            break;
        case 32:
            if (vec) dispatch((jacobi5_v4_kernel<4, 8>), gv, bv, d, st, u, v, nx, ny);
            else dispatch((jacobi5_w_kernel<4, 8>), gv, bv, d, st, u, v, nx, ny);
            break;
        case 64:
            if (vec) dispatch((jacobi5_v4_kernel<4, 16>), gv, bv, d, st, u, v, nx, ny);
            else dispatch((jacobi5_w_kernel<4, 16>), gv, bv, d, st, u, v, nx, ny);
            break;
        }
        hipError_t e = hipGetLastError();
        return e == hipSuccess ? SPMD_OK : hip_fail(e);
    }
    if (BX == 16 && BY == 16 && C <= 4) {
        // Four consecutive logical blocks along x per workgroup (the
        // coarse-grained fetch of Section IV-A, 4 blocks per fetch): their
        // 64 x 16C region runs as 64 x 4 threads with 4C cells each, so
        // every row of the LDS tile is one 256-byte segment instead of four
        // 64-byte ones.  Each cell is computed exactly as in its own block.
        launch_c<64, 4>(4 * C, dim3((c.grid.x + 3) / 4, c.grid.y), d, c.stream, u, v, nx, ny);
    } else if (BX == 16 && BY == 16) launch_c<16, 16>(C, g, d, c.stream, u, v, nx, ny);
    else if (BX == 64 && BY == 1) launch_c<64, 1>(C, g, d, c.stream, u, v, nx, ny);
    else if (BX == 64 && BY == 2) launch_c<64, 2>(C, g, d, c.stream, u, v, nx, ny);
    else if (BX == 32 && BY == 8) launch_c<32, 8>(C, g, d, c.stream, u, v, nx, ny);
    else if (BX == 64 && BY == 4) launch_c<64, 4>(C, g, d, c.stream, u, v, nx, ny);
    else if (BX == 64 && BY == 8) launch_c<64, 8>(C, g, d, c.stream, u, v, nx, ny);
    else if (BX == 128 && BY == 2) launch_c<128, 2>(C, g, d, c.stream, u, v, nx, ny);
    else if (BX == 128 && BY == 4) launch_c<128, 4>(C, g, d, c.stream, u, v, nx, ny);
    else if (BX == 256 && BY == 1) launch_c<256, 1>(C, g, d, c.stream, u, v, nx, ny);
    else return SPMD_ERR_INVALID_DIM;
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SPMD_OK : hip_fail(e);
}

}  // namespace spmd
