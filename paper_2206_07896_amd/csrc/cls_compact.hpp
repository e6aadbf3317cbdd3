// cls_compact.hpp -- tile body of the COMPACT_I32 class: stream compaction
// (a database selection), y = the elements of x greater than t, in order,
// count = how many.
//
// A tile is B threads x I items, B*I consecutive elements; 32-lane warp w
// owns the consecutive segment [w*32*I, (w+1)*32*I) of it.
//   1. local offsets, by warp vote.  A full, 16-byte aligned tile with
//      I >= 4 is read in rows of 32 lanes x 4 elements (16 bytes per lane)
//      and held in registers.  A lane keeps c = 0..4 of its four; the three
//      bit planes of c are balloted over the warp, and popc of each plane
//      below the lane, scaled by 2^plane, is the number kept by the lanes
//      before it.  Rows are chained by their totals.  Other tiles take one
//      element per lane per step (one ballot, popc below the lane), in two
//      passes over the tile (count, then place), so registers do not grow
//      with I.
//   2. warp totals through LDS; barrier; each warp's offset in the tile and
//      the tile's count;
//   3. the tile's offset in y by decoupled look-back over the tiles' counts
//      (the scan class's protocol: tiles start in ticket order);
//   4. before the look-back, every kept element is written to an LDS stage
//      at warp offset + its own (the tile's output, contiguous); after it,
//      the block copies the stage to y at the tile's offset with coalesced
//      stores.
// The last tile writes count.  The pieces below are sequenced by the
// kernel (k_compact.hip), which overlaps one tile's look-back and copy-out
// with the next tile's loads and count.
#pragma once
#include "cls_scan.hpp"

namespace spmd {

template <int B, int I>
struct CompactLds {
    uint32_t warp[B / 32];
    uint32_t excl;
    uint32_t stage[B * I];  // the tile's kept elements, in order
};

// number of lanes below this one in the half-wave whose bit is set in m
__device__ __forceinline__ uint32_t below(uint32_t m) {
    return (uint32_t)__builtin_popcount(m & ((1u << lane32()) - 1u));
}

// A tile between its loads and its stage: the rows it holds in registers
// (rows form only) and each lane's kept-before count per row.
template <int B, int I>
struct CompactFront {
    static constexpr int S = I >= 4 ? I / 4 : 1;
    u32x4 rv[S];
    uint32_t rpos[S];  // kept elements of this warp's segment before this lane's four
    bool rows;         // full, 16-byte aligned tile with I >= 4: the rows form
};

// Issue the tile's loads (rows form); other tiles load in the two passes.
template <int B, int I>
__device__ __forceinline__ void compact_issue(const int32_t* __restrict__ x, uint32_t n, uint32_t tile, bool vec,
                                              CompactFront<B, I>& F) {
    F.rows = false;
    if constexpr (I >= 4) {
        const uint64_t tb = (uint64_t)tile * B * I;
        if (vec && tb + (uint64_t)B * I <= (uint64_t)n) {
            F.rows = true;
            const u32x4* xv = reinterpret_cast<const u32x4*>(x + tb + (uint64_t)(threadIdx.x >> 5) * 32u * I);
#pragma unroll
            for (int q = 0; q < F.S; ++q) F.rv[q] = __builtin_nontemporal_load(xv + q * 32 + lane32());
        }
    }
}

// Step 1: local offsets by warp vote; lane 0 of each warp writes the
// warp's count to LDS (the caller then places a barrier).
template <int B, int I>
__device__ __forceinline__ void compact_count(const int32_t* __restrict__ x, uint32_t n, int32_t t, uint32_t tile,
                                              CompactFront<B, I>& F, CompactLds<B, I>& L) {
    uint32_t run = 0;  // warp-uniform
    if (F.rows) {
#pragma unroll
        for (int q = 0; q < F.S; ++q) {
            const uint32_t c = ((int32_t)F.rv[q].x > t) + ((int32_t)F.rv[q].y > t) + ((int32_t)F.rv[q].z > t) +
                               ((int32_t)F.rv[q].w > t);
            const uint32_t m0 = w32_ballot(c & 1u), m1 = w32_ballot(c & 2u), m2 = w32_ballot(c & 4u);
            F.rpos[q] = run + below(m0) + 2u * below(m1) + 4u * below(m2);
            run += (uint32_t)__builtin_popcount(m0) + 2u * (uint32_t)__builtin_popcount(m1) +
                   4u * (uint32_t)__builtin_popcount(m2);
        }
    } else {
        const uint64_t seg = (uint64_t)tile * B * I + (uint64_t)(threadIdx.x >> 5) * 32u * I;
        for (int k = 0; k < I; ++k) {
            const uint64_t e = seg + (uint64_t)k * 32u + lane32();
            const bool keep = e < (uint64_t)n && x[e] > t;
            run += (uint32_t)__builtin_popcount(w32_ballot(keep));
        }
    }
    if (lane32() == 0) L.warp[threadIdx.x >> 5] = run;
}

// Step 2 (after the barrier): the tile's count and this warp's offset in it.
template <int B, int I>
__device__ __forceinline__ void compact_sums(const CompactLds<B, I>& L, uint32_t& agg, uint32_t& wpre) {
    constexpr int NW = B / 32;
    const uint32_t w = threadIdx.x >> 5;
    agg = 0;
    wpre = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        const uint32_t s = L.warp[k];
        agg += s;
        wpre += ((uint32_t)k < w) ? s : 0u;
    }
}

// Step 4, first half: every kept element to the LDS stage at its offset in
// the tile's output.
template <int B, int I>
__device__ __forceinline__ void compact_stage(const int32_t* __restrict__ x, uint32_t n, int32_t t, uint32_t tile,
                                              uint32_t wpre, const CompactFront<B, I>& F, CompactLds<B, I>& L) {
    if (F.rows) {
#pragma unroll
        for (int q = 0; q < F.S; ++q) {
            uint32_t p = wpre + F.rpos[q];
            const uint32_t v[4] = {F.rv[q].x, F.rv[q].y, F.rv[q].z, F.rv[q].w};
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if ((int32_t)v[j] > t) L.stage[p++] = v[j];
        }
        return;
    }
    const uint64_t seg = (uint64_t)tile * B * I + (uint64_t)(threadIdx.x >> 5) * 32u * I;
    uint32_t p = wpre;  // warp-uniform
    for (int k = 0; k < I; ++k) {
        const uint64_t e = seg + (uint64_t)k * 32u + lane32();
        const int32_t v = e < (uint64_t)n ? x[e] : 0;
        const bool keep = e < (uint64_t)n && v > t;
        const uint32_t m = w32_ballot(keep);
        if (keep) L.stage[p + below(m)] = (uint32_t)v;
        p += (uint32_t)__builtin_popcount(m);
    }
}

}  // namespace spmd
