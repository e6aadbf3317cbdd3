// cls_compact.hpp -- tile body of the COMPACT_I32 class: stream compaction
// (a database selection), y = the elements of x greater than t, in order,
// count = how many.
//
// A tile is B threads x I items, B*I consecutive elements; 32-lane warp w
// owns the consecutive segment [w*32*I, (w+1)*32*I) of it.
//   1. local offsets, by warp vote.  A full, 16-byte aligned tile with
//      I >= 4 is read in rows of 32 lanes x 4 elements (16 bytes per lane).
//      A lane keeps c = 0..4 of its four; the three bit planes of c are
//      balloted over the warp, and popc of each plane below the lane, scaled
//      by 2^plane, is the number kept by the lanes before it.  Rows are
//      chained by their totals.  Other tiles take one element per lane per
//      step: one ballot, popc below the lane.
//   2. warp totals through LDS; barrier; each warp's offset in the tile and
//      the tile's count;
//   3. the tile's offset in y by decoupled look-back over the tiles' counts
//      (the scan class's protocol: tiles start in ticket order);
//   4. before the look-back, every kept element is written to an LDS stage
//      at warp offset + its own (the tile's output, contiguous); after it,
//      the block copies the stage to y at the tile's offset with coalesced
//      stores.
// The last tile writes count.
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

// Warp totals -> this warp's offset in the tile (returned) and the tile's
// count (agg).  Ends with a barrier.
template <int B, int I>
__device__ __forceinline__ uint32_t compact_warp_offset(uint32_t run, uint32_t& agg, CompactLds<B, I>& L) {
    constexpr int NW = B / 32;
    const uint32_t w = threadIdx.x >> 5;
    if (lane32() == 0) L.warp[w] = run;
    __syncthreads();
    uint32_t wpre = 0;
    agg = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        const uint32_t s = L.warp[k];
        agg += s;
        wpre += ((uint32_t)k < w) ? s : 0u;
    }
    return wpre;
}

// The stage is complete: the tile's offset in y by look-back (the last
// tile writes count), then the stage leaves with coalesced stores.
template <int B, int I, typename Hook>
__device__ __forceinline__ void compact_store(int32_t* __restrict__ y, uint32_t* count, uint32_t agg, uint32_t tile,
                                              uint32_t ntiles, uint64_t* status, uint32_t tag, uint32_t* err,
                                              CompactLds<B, I>& L, Hook after_lookback) {
    const uint32_t tid = threadIdx.x;
    if (tid < 64) {
        const uint32_t excl = scan_lookback(status, tile, agg, tag, err);
        if (tid == 0) {
            L.excl = excl;
            if (tile == ntiles - 1) *count = excl + agg;
            after_lookback();
        }
    }
    __syncthreads();  // also orders the stage writes before the reads below
    int32_t* yo = y + L.excl;
    for (uint32_t i = tid; i < agg; i += B) yo[i] = (int32_t)L.stage[i];
}

// Full, 16-byte aligned tile, I >= 4: rows of 32 lanes x 4 elements.
template <int B, int I, typename Hook>
__device__ __forceinline__ void compact_tile_rows(const int32_t* __restrict__ x, int32_t* __restrict__ y,
                                                  uint32_t* count, int32_t t, uint32_t tile, uint32_t ntiles,
                                                  uint64_t* status, uint32_t tag, uint32_t* err,
                                                  CompactLds<B, I>& L, Hook after_lookback) {
    constexpr int S = I / 4;
    const uint64_t seg = (uint64_t)tile * B * I + (uint64_t)(threadIdx.x >> 5) * 32u * I;
    const u32x4* xv = reinterpret_cast<const u32x4*>(x + seg);
    u32x4 rv[S];
    uint32_t rpos[S];  // kept elements of this warp's segment before this lane's four
#pragma unroll
    for (int q = 0; q < S; ++q) rv[q] = __builtin_nontemporal_load(xv + q * 32 + lane32());
    uint32_t run = 0;  // warp-uniform
#pragma unroll
    for (int q = 0; q < S; ++q) {
        const uint32_t c = ((int32_t)rv[q].x > t) + ((int32_t)rv[q].y > t) + ((int32_t)rv[q].z > t) +
                           ((int32_t)rv[q].w > t);
        const uint32_t m0 = w32_ballot(c & 1u), m1 = w32_ballot(c & 2u), m2 = w32_ballot(c & 4u);
        rpos[q] = run + below(m0) + 2u * below(m1) + 4u * below(m2);
        run += (uint32_t)__builtin_popcount(m0) + 2u * (uint32_t)__builtin_popcount(m1) +
               4u * (uint32_t)__builtin_popcount(m2);
    }
    uint32_t agg;
    const uint32_t wpre = compact_warp_offset<B, I>(run, agg, L);
#pragma unroll
    for (int q = 0; q < S; ++q) {
        uint32_t p = wpre + rpos[q];
        const uint32_t v[4] = {rv[q].x, rv[q].y, rv[q].z, rv[q].w};
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if ((int32_t)v[j] > t) L.stage[p++] = v[j];
    }
    compact_store<B, I>(y, count, agg, tile, ntiles, status, tag, err, L, after_lookback);
}

// Any tile: one element per lane per step, one ballot per step, in two
// passes over the tile (count, then place), so registers do not grow with
// I.  Only partial or unaligned tiles take this path.
template <int B, int I, typename Hook>
__device__ __forceinline__ void compact_tile_items(const int32_t* __restrict__ x, int32_t* __restrict__ y,
                                                   uint32_t* count, uint32_t n, int32_t t, uint32_t tile,
                                                   uint32_t ntiles, uint64_t* status, uint32_t tag,
                                                   uint32_t* err, CompactLds<B, I>& L, Hook after_lookback) {
    const uint64_t seg = (uint64_t)tile * B * I + (uint64_t)(threadIdx.x >> 5) * 32u * I;
    uint32_t run = 0;
    for (int k = 0; k < I; ++k) {
        const uint64_t e = seg + (uint64_t)k * 32u + lane32();
        const bool keep = e < (uint64_t)n && x[e] > t;
        run += (uint32_t)__builtin_popcount(w32_ballot(keep));
    }
    uint32_t agg;
    uint32_t p = compact_warp_offset<B, I>(run, agg, L);  // warp-uniform
    for (int k = 0; k < I; ++k) {
        const uint64_t e = seg + (uint64_t)k * 32u + lane32();
        const int32_t v = e < (uint64_t)n ? x[e] : 0;
        const bool keep = e < (uint64_t)n && v > t;
        const uint32_t m = w32_ballot(keep);
        if (keep) L.stage[p + below(m)] = (uint32_t)v;
        p += (uint32_t)__builtin_popcount(m);
    }
    compact_store<B, I>(y, count, agg, tile, ntiles, status, tag, err, L, after_lookback);
}

// Thread 0 calls `after_lookback` once the tile's inclusive count is
// published (no other tile can wait on this one any more).
template <int B, int I, typename Hook>
__device__ __forceinline__ void compact_tile(const int32_t* __restrict__ x, int32_t* __restrict__ y,
                                             uint32_t* count, uint32_t n, int32_t t, uint32_t tile,
                                             uint32_t ntiles, uint64_t* status, uint32_t tag, uint32_t* err,
                                             bool vec, CompactLds<B, I>& L, Hook after_lookback) {
    if constexpr (I >= 4) {
        if (vec && (uint64_t)tile * B * I + (uint64_t)B * I <= (uint64_t)n) {
            compact_tile_rows<B, I>(x, y, count, t, tile, ntiles, status, tag, err, L, after_lookback);
            return;
        }
    }
    compact_tile_items<B, I>(x, y, count, n, t, tile, ntiles, status, tag, err, L, after_lookback);
}

}  // namespace spmd
