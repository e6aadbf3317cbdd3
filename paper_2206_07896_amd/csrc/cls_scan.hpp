// cls_scan.hpp -- tile body of the SCAN_I32 class (inclusive prefix sum
// modulo 2^32).
//
// A tile is B threads x I consecutive items per thread:
//   1. thread-serial inclusive scan of its I items (registers);
//   2. 32-lane inclusive scan of the thread totals (warp32 DPP scan);
//   3. the last lane of each warp writes the warp total to LDS; barrier;
//      each thread adds the totals of the warps before its own;
//   4. grid carry by decoupled look-back (Merrill and Garland, "Single-pass
//      Parallel Prefix Scan with Decoupled Look-back", 2016): the tile
//      publishes its aggregate, wave 0 reads the status words of up to 64
//      predecessors at a time, sums aggregates back to the nearest inclusive
//      prefix, and publishes its own inclusive prefix; barrier;
//   5. every item gets carry + warp prefix + thread prefix.
// Tiles must start in index order (a ticket or an ordered queue hands the
// indices out), so every predecessor a tile waits for has already started
// and the waits end.  Each wait is still bounded: past the spin limit the
// tile flags the device error word and stops waiting.
//
// Status words (warp32.hpp) carry flag 1 = aggregate, 2 = inclusive prefix.
#pragma once
#include "common.hpp"
#include "warp32.hpp"

namespace spmd {

constexpr uint32_t SCAN_AGG = 1u, SCAN_INCL = 2u;
constexpr uint32_t LOOKBACK_SPIN_LIMIT = 1u << 22;

template <int B>
struct ScanLds {
    uint32_t warp[B / 32];
    uint32_t excl;
};

// Exclusive carry of `tile`, computed by wave 0 (the 64 lanes call it).
// Polling is the costly part on gfx950: every status read is a device-
// coherent access, and many tiles poll the same few lines.  So the wave
// first polls only the immediate predecessor (one address for all lanes,
// exponential back-off) until it has published; older predecessors have
// almost always published by then.  It then reads 64 predecessors at a
// time, waits (with back-off) for any lane still unwritten, keeps the words
// up to the nearest inclusive prefix, and moves back 64 if there is none.
__device__ __forceinline__ uint32_t scan_lookback(uint64_t* status, uint32_t tile, uint32_t agg, uint32_t tag,
                                                  uint32_t* err) {
    const uint32_t lane = lane64();
    if (tile == 0) {
        if (lane == 0) status_put(status, status_pack(agg, SCAN_INCL, tag));
        return 0;
    }
    if (lane == 0) status_put(status + tile, status_pack(agg, SCAN_AGG, tag));
    uint32_t spins = 0, nap = 1;
    while (status_flag(status_get(status + tile - 1), tag) == 0u) {
        if (++spins >= LOOKBACK_SPIN_LIMIT) break;  // the window loop below reports it
        backoff_sleep(nap);
        nap = nap < 16u ? nap * 2u : 16u;
    }
    uint32_t excl = 0;
    int64_t pos = (int64_t)tile - 1;
    for (;;) {
        const int64_t idx = pos - (int64_t)lane;
        uint64_t s = 0;
        uint32_t f = SCAN_INCL;  // before tile 0: a zero prefix
        spins = 0;
        nap = 1;
        for (;;) {
            if (idx >= 0) {
                s = status_get(status + idx);
                f = status_flag(s, tag);
            }
            if (__builtin_amdgcn_ballot_w64(f == 0u) == 0) break;
            if (++spins >= LOOKBACK_SPIN_LIMIT) {
                if (lane == 0) atomicOr(err, ERRBIT_SPIN_LIMIT);
                if (f == 0u) {
                    s = 0;
                    f = SCAN_INCL;
                }
                break;
            }
            backoff_sleep(nap);
            nap = nap < 16u ? nap * 2u : 16u;
        }
        const uint64_t incl = __builtin_amdgcn_ballot_w64(f == SCAN_INCL);
        const uint32_t val = (uint32_t)(s >> 32);
        if (incl) {
            const uint32_t k = (uint32_t)__builtin_ctzll(incl);  // nearest inclusive predecessor
            excl += wave_sum(lane <= k ? val : 0u);
            break;
        }
        excl += wave_sum(val);
        pos -= 64;
    }
    if (lane == 0) status_put(status + tile, status_pack(excl + agg, SCAN_INCL, tag));
    return excl;
}

// Scan tile `tile` of x into y.  The caller places a barrier before the LDS
// area is reused.
template <int B, int I>
__device__ __forceinline__ void scan_tile(const int32_t* __restrict__ x, int32_t* __restrict__ y, uint32_t n,
                                          uint32_t tile, uint64_t* status, uint32_t tag, uint32_t* err, bool vec,
                                          ScanLds<B>& L) {
    constexpr uint64_t T = (uint64_t)B * I;
    constexpr int NW = B / 32;
    const uint32_t t = threadIdx.x;
    const uint64_t base = (uint64_t)tile * T + (uint64_t)t * I;
    const bool full = base + I <= (uint64_t)n;
    uint32_t v[I];
    if constexpr (I % 4 == 0) {
        if (vec && full) {
            const u32x4* xv = reinterpret_cast<const u32x4*>(x + base);
#pragma unroll
            for (int q = 0; q < I / 4; ++q) {
                u32x4 a = __builtin_nontemporal_load(xv + q);
                v[4 * q] = a.x;
                v[4 * q + 1] = a.y;
                v[4 * q + 2] = a.z;
                v[4 * q + 3] = a.w;
            }
        } else {
#pragma unroll
            for (int k = 0; k < I; ++k) v[k] = (base + k < n) ? (uint32_t)x[base + k] : 0u;
        }
    } else {
#pragma unroll
        for (int k = 0; k < I; ++k) v[k] = (base + k < n) ? (uint32_t)x[base + k] : 0u;
    }
#pragma unroll
    for (int k = 1; k < I; ++k) v[k] += v[k - 1];
    const uint32_t tot = v[I - 1];
    const uint32_t wincl = w32_inclusive_add(tot);
    if ((t & 31u) == 31u) L.warp[t >> 5] = wincl;
    __syncthreads();
    uint32_t wpre = 0, agg = 0;
    const uint32_t mywarp = t >> 5;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const uint32_t s = L.warp[w];
        agg += s;
        wpre += ((uint32_t)w < mywarp) ? s : 0u;
    }
    if (t < 64) {
        const uint32_t excl = scan_lookback(status, tile, agg, tag, err);
        if (t == 0) L.excl = excl;
    }
    __syncthreads();
    const uint32_t pre = L.excl + wpre + (wincl - tot);
    if constexpr (I % 4 == 0) {
        if (vec && full) {
            u32x4* yv = reinterpret_cast<u32x4*>(y + base);
#pragma unroll
            for (int q = 0; q < I / 4; ++q) {
                u32x4 a;
                a.x = pre + v[4 * q];
                a.y = pre + v[4 * q + 1];
                a.z = pre + v[4 * q + 2];
                a.w = pre + v[4 * q + 3];
                __builtin_nontemporal_store(a, yv + q);
            }
            return;
        }
    }
#pragma unroll
    for (int k = 0; k < I; ++k)
        if (base + k < n) y[base + k] = (int32_t)(pre + v[k]);
}

}  // namespace spmd
