// cls_reduce.hpp -- block body of the REDUCE_I32 class.
//
// One logical block of B threads sums its segment x[lo, hi) into one
// partial; the block that takes the last completion ticket then sums all G
// partials into *out and re-arms the ticket counter.
//
// gfx950 mapping of the block tree: levels whose stride is >= 64 combine
// values held by different waves and go through LDS with a barrier; levels
// with stride < 64 combine lanes of one wave and run as a register
// butterfly inside the wave (no barrier is needed between lanes of one
// wave).  Integer addition modulo 2^32 is associative and commutative, so
// any tree shape gives the same bits.
#pragma once
#include "warp32.hpp"

namespace spmd {

template <int B>
struct ReduceLds {
    uint32_t wave[B / 64];
    uint32_t last;
};

// Sum of v over the block; valid in thread 0 only.  Ends with a barrier so
// the LDS slots may be reused.
template <int B>
__device__ __forceinline__ uint32_t block_sum_t0(uint32_t v, ReduceLds<B>& L) {
    constexpr int NW = B / 64;
    uint32_t w = wave_sum(v);
    if (lane64() == 0) L.wave[threadIdx.x / 64] = w;
    __syncthreads();
    uint32_t tot = 0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NW; ++i) tot += L.wave[i];
    }
    __syncthreads();
    return tot;
}

// Thread t's share of x[lo, hi): element j with j - lo = t (mod B); four
// 16-byte loads in flight per step when x + lo is 16-byte aligned.
template <int B>
__device__ __forceinline__ uint32_t segment_sum(const int32_t* __restrict__ x, uint64_t lo, uint64_t hi, bool vec) {
    const uint32_t t = threadIdx.x;
    uint32_t acc = 0;
    if (lo >= hi) return 0;
    if (vec) {
        const u32x4* xv = reinterpret_cast<const u32x4*>(x + lo);
        const uint64_t nv = (hi - lo) >> 2;
        uint64_t k = t;
        for (; k + 3 * B < nv; k += 4 * B) {
            u32x4 a = __builtin_nontemporal_load(xv + k);
            u32x4 b = __builtin_nontemporal_load(xv + k + B);
            u32x4 c = __builtin_nontemporal_load(xv + k + 2 * B);
            u32x4 d = __builtin_nontemporal_load(xv + k + 3 * B);
            acc += (a.x + a.y) + (a.z + a.w) + (b.x + b.y) + (b.z + b.w);
            acc += (c.x + c.y) + (c.z + c.w) + (d.x + d.y) + (d.z + d.w);
        }
        for (; k < nv; k += B) {
            u32x4 a = __builtin_nontemporal_load(xv + k);
            acc += (a.x + a.y) + (a.z + a.w);
        }
        for (uint64_t j = lo + (nv << 2) + t; j < hi; j += B) acc += (uint32_t)x[j];
    } else {
        for (uint64_t j = lo + t; j < hi; j += B) acc += (uint32_t)x[j];
    }
    return acc;
}

// One logical block `bid` of a G-block reduction.
template <int B>
__device__ __forceinline__ void reduce_block(const int32_t* __restrict__ x, int32_t* partials, int32_t* out,
                                             uint32_t n, uint32_t seg, uint32_t G, uint32_t bid,
                                             uint32_t* counter, bool vec, ReduceLds<B>& L) {
    const uint64_t lo = (uint64_t)bid * seg;
    const uint64_t hi = lo + seg < (uint64_t)n ? lo + seg : (uint64_t)n;
    uint32_t tot = block_sum_t0<B>(segment_sum<B>(x, lo, hi, vec), L);
    if (threadIdx.x == 0) {
        partials[bid] = (int32_t)tot;
        fence_dev();  // the partial is visible before the ticket is taken
        uint32_t ticket = atomic_add_dev(counter, 1u);
        L.last = (ticket == G - 1u) ? 1u : 0u;
    }
    __syncthreads();
    const bool last = L.last != 0u;
    __syncthreads();
    if (!last) return;
    fence_dev();  // acquire the other blocks' partials
    uint32_t acc = 0;
    for (uint32_t j = threadIdx.x; j < G; j += B)
        acc += __hip_atomic_load(reinterpret_cast<uint32_t*>(partials) + j, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
    uint32_t total = block_sum_t0<B>(acc, L);
    if (threadIdx.x == 0) {
        *out = (int32_t)total;
        store_release_dev(counter, 0u);  // re-arm for the next launch
    }
}

}  // namespace spmd
