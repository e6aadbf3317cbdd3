// k_warptest.hip -- WARPTEST (32-lane warp-operation conformance) and
// REVERSE_I32 (the paper's dynamic-shared-memory example).
#include "common.hpp"
#include "warp32.hpp"

namespace spmd {

__device__ __forceinline__ int warp_op_rt(int op, int v, uint32_t p, uint32_t w) {
    switch (op) {
    case 0: return w32_shfl(v, p, w);
    case 1: return w32_shfl_up(v, p, w);
    case 2: return w32_shfl_down(v, p, w);
    default: return w32_shfl_xor(v, p, w);
    }
}

// Compile-time forms.  Full-width butterflies use ds_swizzle; the others
// use the generic permute with constant operands.
template <int OP, int P, int W>
__device__ __forceinline__ int warp_op_ct(int v) {
    if constexpr (OP == 0) return w32_shfl_up(v, P, W);
    else if constexpr (OP == 1) return w32_shfl_down(v, P, W);
    else if constexpr (OP == 2) {
        if constexpr (W == 32) return w32_xor_c<P>(v);
        else return w32_shfl_xor(v, P, W);
    } else return w32_shfl(v, P, W);
}

template <int OP, int WS>
__device__ __forceinline__ void ct_group(int v, int32_t* out, uint64_t total, uint64_t gtid) {
    constexpr int W = 32 >> WS;
    constexpr int base = 864 + (OP * 2 + WS) * 5;
    out[(uint64_t)(base + 0) * total + gtid] = warp_op_ct<OP, 1, W>(v);
    out[(uint64_t)(base + 1) * total + gtid] = warp_op_ct<OP, 2, W>(v);
    out[(uint64_t)(base + 2) * total + gtid] = warp_op_ct<OP, 4, W>(v);
    out[(uint64_t)(base + 3) * total + gtid] = warp_op_ct<OP, 8, W>(v);
    out[(uint64_t)(base + 4) * total + gtid] = warp_op_ct<OP, 16, W>(v);
}

__global__ void warptest_kernel(const int32_t* __restrict__ val, const uint32_t* __restrict__ pred,
                                int32_t* __restrict__ out) {
    const uint64_t total = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t gtid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int v = val[gtid];
    const uint32_t pr = pred[gtid];
    for (int c = 0; c < 768; ++c) {
        const int op = c / 192;
        const uint32_t w = 1u << ((c / 32) % 6);
        const uint32_t p = (uint32_t)(c % 32);
        out[(uint64_t)c * total + gtid] = warp_op_rt(op, v, p, w);
    }
    for (int c = 768; c < 864; ++c) {
        const int vote = (c - 768) / 32;
        const bool bit = (pr >> ((c - 768) % 32)) & 1u;
        const uint32_t b = w32_ballot(bit);
        int32_t r;
        if (vote == 0) r = (int32_t)b;
        else if (vote == 1) r = b != 0u ? 1 : 0;
        else r = b == 0xFFFFFFFFu ? 1 : 0;
        out[(uint64_t)c * total + gtid] = r;
    }
    ct_group<0, 0>(v, out, total, gtid);
    ct_group<0, 1>(v, out, total, gtid);
    ct_group<1, 0>(v, out, total, gtid);
    ct_group<1, 1>(v, out, total, gtid);
    ct_group<2, 0>(v, out, total, gtid);
    ct_group<2, 1>(v, out, total, gtid);
    ct_group<3, 0>(v, out, total, gtid);
    ct_group<3, 1>(v, out, total, gtid);
}

int launch_warptest(const LaunchCtx& c) {
    if (c.block.x % 32 != 0 || c.block.y != 1 || c.block.z != 1 || c.grid.y != 1 || c.grid.z != 1)
        return SPMD_ERR_INVALID_DIM;
    auto val = arg<const int32_t*>(c.args, 0);
    auto pred = arg<const uint32_t*>(c.args, 1);
    auto out = arg<int32_t*>(c.args, 2);
    if (!val || !pred || !out) return SPMD_ERR_ARGS;
    dispatch(warptest_kernel, dim3(c.grid.x), dim3(c.block.x), c.dyn_shmem, c.stream, val, pred, out);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SPMD_OK : hip_fail(e);
}

// The paper's dynamicReverse: s is the block's dynamic shared memory.
__global__ void reverse_i32_kernel(int32_t* d, uint32_t n) {
    extern __shared__ int32_t s[];
    const uint32_t t = threadIdx.x;
    const uint32_t tr = n - t - 1u;
    s[t] = d[t];
    __syncthreads();
    d[t] = s[tr];
}

int launch_reverse_i32(const LaunchCtx& c) {
    auto d = arg<int32_t*>(c.args, 0);
    auto n = arg<uint32_t>(c.args, 1);
    if (!d) return SPMD_ERR_ARGS;
    if (c.grid.x != 1 || c.grid.y != 1 || c.grid.z != 1 || c.block.y != 1 || c.block.z != 1 || c.block.x != n)
        return SPMD_ERR_INVALID_DIM;
    if (c.dyn_shmem < 4ull * n) return SPMD_ERR_SHMEM;
    dispatch(reverse_i32_kernel, dim3(1), dim3(n), c.dyn_shmem, c.stream, d, n);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SPMD_OK : hip_fail(e);
}

}  // namespace spmd
