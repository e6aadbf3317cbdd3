// cls_hist.hpp -- block body of the HIST256_U32 class.
//
// Phase 1: zero the block's LDS sub-histograms; barrier.
// Phase 2: every key adds 1 to bin (key & 255) of an LDS sub-histogram with
//          an LDS atomic; barrier.
// Phase 3: each non-zero bin, summed over the block's copies, goes to the
//          global histogram with one device-scope atomic add.
//
// gfx950 detail: LDS atomics of one wave to the same address serialise, and
// skewed keys (a Zipf law puts a fifth of all keys in one bin) make that the
// bottleneck.  Lanes therefore spread over COPIES sub-histograms by lane
// index (lane % COPIES), each padded to 257 words so the copies of one bin
// sit in different LDS banks.  The counts are exact, so the split changes
// nothing in the result.
#pragma once
#include "common.hpp"
#include "warp32.hpp"

namespace spmd {

constexpr int HIST_STRIDE = 257;
constexpr int HIST_COPIES = 4;

template <int COPIES>
struct HistLds {
    uint32_t s[COPIES * HIST_STRIDE];
};

template <int B, int COPIES>
__device__ __forceinline__ void hist_block(const uint32_t* __restrict__ keys, uint32_t* hist, uint64_t lo,
                                           uint64_t hi, bool vec, HistLds<COPIES>& L) {
    const uint32_t t = threadIdx.x;
    for (uint32_t i = t; i < COPIES * HIST_STRIDE; i += B) L.s[i] = 0u;
    __syncthreads();
    uint32_t* mine = L.s + (lane64() % COPIES) * HIST_STRIDE;
    auto add = [&](uint32_t k) {
        __hip_atomic_fetch_add(mine + (k & 255u), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    if (lo < hi) {
        if (vec) {
            const u32x4* kv = reinterpret_cast<const u32x4*>(keys + lo);
            const uint64_t nv = (hi - lo) >> 2;
            uint64_t k = t;
            for (; k + B < nv; k += 2 * B) {
                u32x4 a = __builtin_nontemporal_load(kv + k);
                u32x4 b = __builtin_nontemporal_load(kv + k + B);
                add(a.x); add(a.y); add(a.z); add(a.w);
                add(b.x); add(b.y); add(b.z); add(b.w);
            }
            for (; k < nv; k += B) {
                u32x4 a = __builtin_nontemporal_load(kv + k);
                add(a.x); add(a.y); add(a.z); add(a.w);
            }
            for (uint64_t j = lo + (nv << 2) + t; j < hi; j += B) add(keys[j]);
        } else {
            for (uint64_t j = lo + t; j < hi; j += B) add(keys[j]);
        }
    }
    __syncthreads();
    for (uint32_t bin = t; bin < 256u; bin += B) {
        uint32_t c = 0;
#pragma unroll
        for (int r = 0; r < COPIES; ++r) c += L.s[r * HIST_STRIDE + bin];
        if (c) __hip_atomic_fetch_add(hist + bin, c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

}  // namespace spmd
