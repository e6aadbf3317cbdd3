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
#include "common.hpp"
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

constexpr uint32_t REDUCE_SPIN_LIMIT = 1u << 22;

// One logical block `bid` of a G-block reduction.  Cross-block state
// (`ctl`, `status`): ctl[0] is the completion ticket, status[b] the partial
// of block b as a tagged status word.  Thread 0 publishes the block's
// partial (to `partials`, when given, and as a status word), then takes a
// ticket; the block holding ticket G-1 reads the G status words (waiting,
// boundedly, for any not yet visible), sums them, writes *out, clears the
// status words and re-arms the ticket, so the next launch finds the state
// as the first one did.  Returns true in the block that finished.
template <int B>
__device__ __forceinline__ bool reduce_block(const int32_t* __restrict__ x, int32_t* partials, int32_t* out,
                                             uint32_t n, uint32_t seg, uint32_t G, uint32_t bid, uint32_t* ctl,
                                             uint64_t* status, uint32_t tag, uint32_t* err, bool vec,
                                             ReduceLds<B>& L) {
    const uint64_t lo = (uint64_t)bid * seg;
    const uint64_t hi = lo + seg < (uint64_t)n ? lo + seg : (uint64_t)n;
    const uint32_t tot = block_sum_t0<B>(segment_sum<B>(x, lo, hi, vec), L);
    if (threadIdx.x == 0) {
        if (partials) partials[bid] = (int32_t)tot;
        status_put(status + bid, status_pack(tot, 1u, tag));
        L.last = (atomic_add_dev(ctl, 1u) == G - 1u) ? 1u : 0u;
    }
    __syncthreads();
    const bool last = L.last != 0u;
    __syncthreads();
    if (!last) return false;
    // The G status words, eight independent loads in flight per thread;
    // only words not yet visible are polled again.
    uint32_t acc = 0;
    for (uint32_t j0 = threadIdx.x; j0 < G; j0 += 8u * B) {
        uint64_t w[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const uint32_t j = j0 + (uint32_t)q * B;
            w[q] = j < G ? status_get(status + j) : status_pack(0u, 1u, tag);
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const uint32_t j = j0 + (uint32_t)q * B;
            for (uint32_t spins = 0; status_flag(w[q], tag) == 0u; ++spins) {
                if (spins >= REDUCE_SPIN_LIMIT) {
                    atomicOr(err, ERRBIT_SPIN_LIMIT);
                    w[q] = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                w[q] = status_get(status + j);
            }
            acc += (uint32_t)(w[q] >> 32);
        }
    }
    const uint32_t total = block_sum_t0<B>(acc, L);
    // Every other block has published and returned: clear the status words
    // and re-arm the ticket for the next launch.
    for (uint32_t j = threadIdx.x; j < G; j += B) status_put(status + j, 0ull);
    if (threadIdx.x == 0) {
        *out = (int32_t)total;
        put_dev(ctl, 0u);
    }
    return true;
}

}  // namespace spmd
