// cls_hist.hpp -- block body of the HIST256_U32 class.
//
// Phase 1: zero the block's LDS sub-histograms; barrier.
// Phase 2: every key adds 1 to bin (key & 255) of an LDS sub-histogram with
//          an LDS atomic; barrier.
// Phase 3: each non-zero bin, summed over the block's copies, goes to the
//          global histogram with one device-scope atomic add.
//
// gfx950 detail: LDS atomics of one wave to the same address serialise, and
// skewed keys (bounded Zipf puts a fifth of all keys in one bin at exponent
// 1.1, three fifths at 2) make that the bottleneck.  Two measures:
//   * lanes spread over COPIES sub-histograms by lane index (lane % COPIES),
//     each padded to 257 words so the copies of one bin sit in different
//     LDS banks;
//   * a wave keeps a candidate hot bin.  Once per eight keys per lane it
//     votes on it; when HOT_LANES or more lanes hold it, the eight keys go
//     through the vote path -- the lanes holding the hot bin drop out and
//     the first of them adds their number (popc of the ballot) in one
//     atomic -- otherwise through plain atomics, and the candidate is
//     replaced by the first lane's key (a fresh draw from the key law, so a
//     hot bin is found quickly).  Unskewed keys pay one ballot per eight
//     keys; under heavy skew the longest chain of same-address atomics
//     collapses to one.
// The loads of the next eight keys are issued before the current ones are
// counted, so twice the bytes are in flight.  Counts are exact, so none of
// this changes the result.
#pragma once
#include "common.hpp"
#include "warp32.hpp"

namespace spmd {

constexpr int HIST_STRIDE = 257;
constexpr int HIST_COPIES = 4;
constexpr uint32_t HIST_HOT_LANES = 16;

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
    auto plain = [&](uint32_t k) {
        __hip_atomic_fetch_add(mine + (k & 255u), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    auto voted = [&](uint32_t k, uint32_t hot) {
        const uint32_t b = k & 255u;
        const uint64_t same = __builtin_amdgcn_ballot_w64(b == hot);
        uint32_t v = 1u;
        if (b == hot) v = lane64() == (uint32_t)__builtin_ctzll(same) ? (uint32_t)__builtin_popcountll(same) : 0u;
        if (v) __hip_atomic_fetch_add(mine + b, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    // Candidate hot bin; 256 matches no key.  Lanes leave the loop below at
    // different trips, so each vote reads the first active lane's candidate:
    // a vote is only exact when every active lane compares with the same
    // bin, and that is all it needs.
    uint32_t hot = 256u;
    auto count8 = [&](u32x4 a, u32x4 b) {
        const uint32_t h = __builtin_amdgcn_readfirstlane(hot);
        const uint64_t m = __builtin_amdgcn_ballot_w64((a.x & 255u) == h);
        if ((uint32_t)__builtin_popcountll(m) >= HIST_HOT_LANES) {
            voted(a.x, h); voted(a.y, h); voted(a.z, h); voted(a.w, h);
            voted(b.x, h); voted(b.y, h); voted(b.z, h); voted(b.w, h);
        } else {
            hot = __builtin_amdgcn_readfirstlane(a.x & 255u);
            plain(a.x); plain(a.y); plain(a.z); plain(a.w);
            plain(b.x); plain(b.y); plain(b.z); plain(b.w);
        }
    };
    if (lo < hi) {
        if (vec) {
            const u32x4* kv = reinterpret_cast<const u32x4*>(keys + lo);
            const uint64_t nv = (hi - lo) >> 2;
            uint64_t k = t;
            if (k + B < nv) {
                u32x4 a = __builtin_nontemporal_load(kv + k);
                u32x4 b = __builtin_nontemporal_load(kv + k + B);
                for (; k + 3 * B < nv; k += 2 * B) {
                    const u32x4 c = __builtin_nontemporal_load(kv + k + 2 * B);
                    const u32x4 d = __builtin_nontemporal_load(kv + k + 3 * B);
                    count8(a, b);
                    a = c;
                    b = d;
                }
                count8(a, b);
                k += 2 * B;
            }
            for (; k < nv; k += B) {
                const u32x4 a = __builtin_nontemporal_load(kv + k);
                plain(a.x); plain(a.y); plain(a.z); plain(a.w);
            }
            for (uint64_t j = lo + (nv << 2) + t; j < hi; j += B) plain(keys[j]);
        } else {
            for (uint64_t j = lo + t; j < hi; j += B) plain(keys[j]);
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
