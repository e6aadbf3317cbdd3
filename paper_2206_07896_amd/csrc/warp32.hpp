// warp32.hpp -- CUDA's 32-lane warp operations on gfx950's 64-lane waves.
//
// A CUDA warp is 32 threads; a gfx950 wavefront is 64 lanes.  Thread t of a
// block is lane t % 64 of wave t / 64, so CUDA warp w = t / 32 is the lower
// (w even) or upper (w odd) half of wave w / 2.  Every operation here keeps
// its effects inside the caller's half-wave, which is exactly CUDA warp
// semantics for full masks:
//   shfl(v, s, w)      : v of lane seg + (s mod w)
//   shfl_up(v, d, w)   : i <  d     ? own : v of lane - d
//   shfl_down(v, d, w) : i + d >= w ? own : v of lane + d
//   shfl_xor(v, m, w)  : lane i^m if it is not in a later segment, else own
//   ballot(p)          : 32-bit mask of the half-wave's predicates
// with i = lane % w and seg = the first lane of the caller's w-segment.  The
// parameter is taken modulo 32.
//
// Mechanisms:
//  - ds_bpermute (any source lane of the 64) for runtime parameters;
//  - ds_swizzle in bit mode (and 0x1F, xor m) for butterflies with a
//    compile-time mask: it never leaves a 32-lane group;
//  - DPP row_shr / row_bcast:15 for the inclusive add-scan: row operations
//    stay within 16-lane rows, and row_bcast:15 with row mask 0xA feeds row
//    0 into row 1 and row 2 into row 3, never across the two halves.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spmd {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t lane64() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
__device__ __forceinline__ uint32_t lane32() { return lane64() & 31u; }

__device__ __forceinline__ int bperm(uint32_t src_lane, int v) {
    return __builtin_amdgcn_ds_bpermute((int)(src_lane << 2), v);
}

__device__ __forceinline__ int w32_shfl(int v, uint32_t src, uint32_t width) {
    uint32_t l = lane64();
    uint32_t seg = l & ~(width - 1u);  // width divides 32, so seg stays in the half
    return bperm(seg + (src & (width - 1u)), v);
}

__device__ __forceinline__ int w32_shfl_up(int v, uint32_t d, uint32_t width) {
    uint32_t l = lane64();
    d &= 31u;
    uint32_t i = l & (width - 1u);
    return bperm(i >= d ? l - d : l, v);
}

__device__ __forceinline__ int w32_shfl_down(int v, uint32_t d, uint32_t width) {
    uint32_t l = lane64();
    d &= 31u;
    uint32_t i = l & (width - 1u);
    return bperm(i + d < width ? l + d : l, v);
}

__device__ __forceinline__ int w32_shfl_xor(int v, uint32_t m, uint32_t width) {
    uint32_t l = lane64();
    uint32_t h = l & 32u, i = l & 31u;
    uint32_t j = i ^ (m & 31u);
    uint32_t last = i | (width - 1u);  // last lane of the caller's segment
    return bperm(j <= last ? h + j : l, v);
}

__device__ __forceinline__ uint32_t w32_ballot(bool p) {
    uint64_t b = __builtin_amdgcn_ballot_w64(p);
    return (uint32_t)(b >> (lane64() & 32u));
}
__device__ __forceinline__ bool w32_any(bool p) { return w32_ballot(p) != 0u; }
__device__ __forceinline__ bool w32_all(bool p) { return w32_ballot(p) == 0xFFFFFFFFu; }

// Butterfly with a compile-time mask M < 32 at full width (ds_swizzle,
// bit mode: and_mask 0x1F, or_mask 0, xor_mask M).
template <int M>
__device__ __forceinline__ int w32_xor_c(int v) {
    static_assert(M > 0 && M < 32, "mask");
    return __builtin_amdgcn_ds_swizzle(v, (M << 10) | 0x1F);
}

// Inclusive add-scan over each 32-lane half (DPP).  Rows are 16 lanes:
// shr 1, 2, 4, 8 scan each row; row_bcast:15 then adds the total of rows 0
// and 2 (lane 15 and lane 47) into rows 1 and 3.
__device__ __forceinline__ uint32_t w32_inclusive_add(uint32_t v) {
    int x = (int)v;
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xF, 0xF, false);  // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xF, 0xF, false);  // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xF, 0xF, false);  // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xF, 0xF, false);  // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xA, 0xF, false);  // row_bcast:15, rows 1 and 3
    return (uint32_t)x;
}

// Sum over each 32-lane half, result in every lane of the half.
__device__ __forceinline__ uint32_t w32_sum(uint32_t v) {
    int x = (int)v;
    x += w32_xor_c<1>(x);
    x += w32_xor_c<2>(x);
    x += w32_xor_c<4>(x);
    x += w32_xor_c<8>(x);
    x += w32_xor_c<16>(x);
    return (uint32_t)x;
}

// Sum over the whole 64-lane wave, result in every lane.
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
    uint32_t s = w32_sum(v);
    return (uint32_t)__builtin_amdgcn_readlane((int)s, 0) + (uint32_t)__builtin_amdgcn_readlane((int)s, 32);
}

// Cross-block protocols (tickets, look-back and partial-sum status words,
// queue cursors) use only relaxed device-scope atomics.  On gfx950 these
// are performed at the device coherence point (sc1) and need no cache
// maintenance, whereas acquire/release at device scope writes back and
// invalidates the whole L2 of the issuing XCD on every use.  No protocol
// here needs such fences: every value a block hands to another block
// travels inside the same 64-bit atomic word as its ready flag.
__device__ __forceinline__ uint32_t atomic_add_dev(uint32_t* p, uint32_t v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t load_dev(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void put_dev(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t atomic_add_dev64(uint64_t* p, uint64_t v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t status_get(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void status_put(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A status word is (value << 32) | (tag << 2) | flag, flag in 1..3.  A word
// whose 30-bit tag differs from the reader's tag reads as "not written", so
// arrays of status words need no clearing between uses with different tags.
__device__ __forceinline__ uint64_t status_pack(uint32_t v, uint32_t flag, uint32_t tag) {
    return ((uint64_t)v << 32) | ((uint64_t)(tag & 0x3FFFFFFFu) << 2) | flag;
}
__device__ __forceinline__ uint32_t status_flag(uint64_t s, uint32_t tag) {
    return (((uint32_t)s >> 2) == (tag & 0x3FFFFFFFu)) ? ((uint32_t)s & 3u) : 0u;
}

// Back-off between polls of a status word: `k` sleeps of 64 cycles.
__device__ __forceinline__ void backoff_sleep(uint32_t k) {
    for (uint32_t i = 0; i < k; ++i) __builtin_amdgcn_s_sleep(1);
}

}  // namespace spmd
