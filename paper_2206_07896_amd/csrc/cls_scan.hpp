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

template <int B, int I>
struct ScanLds {
    uint32_t warp[B / 32];
    uint32_t excl;
    // Tile staging for I >= 4: the tile travels between HBM and registers
    // through LDS so that global loads and stores are fully coalesced
    // (lane-consecutive 16-byte chunks) while each thread still owns I
    // consecutive items.
    alignas(16) uint32_t tile[I >= 4 ? B * I : 4];
};

// LDS slot of 16-byte chunk c of a staged tile with S chunks per thread:
// c ^ ((c / S) mod 8).  It permutes chunks within aligned groups of eight,
// so that both the striped pass (lanes take consecutive chunks) and the
// blocked pass (lane t takes chunks t*S .. t*S+S-1) touch eight distinct
// slots per eight lanes: no LDS bank conflicts either way.
template <int S>
__device__ __forceinline__ uint32_t stage_slot(uint32_t c) {
    if constexpr (S >= 2) return c ^ ((c / S) & 7u);
    else return c;
}

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

struct NoHook {
    __device__ void operator()() const {}
};

// Scan tile `tile` of x into y.  The caller places a barrier before the LDS
// area is reused.  Thread 0 calls `after_lookback` once the tile's
// inclusive prefix is published, i.e. once no other tile can wait on this
// one any more.
template <int B, int I, typename Hook = NoHook>
__device__ __forceinline__ void scan_tile(const int32_t* __restrict__ x, int32_t* __restrict__ y, uint32_t n,
                                          uint32_t tile, uint64_t* status, uint32_t tag, uint32_t* err, bool vec,
                                          ScanLds<B, I>& L, Hook after_lookback = Hook()) {
    constexpr uint64_t T = (uint64_t)B * I;
    constexpr int NW = B / 32;
    constexpr int S = I / 4;  // 16-byte chunks per thread
    const uint32_t t = threadIdx.x;
    const uint64_t tbase = (uint64_t)tile * T;
    const uint64_t base = tbase + (uint64_t)t * I;
    // a full, aligned tile is staged through LDS; the rest is read directly
    bool staged = false;
    if constexpr (I >= 4) staged = vec && tbase + T <= (uint64_t)n;
    uint32_t v[I];
    if constexpr (I >= 4) {
        if (staged) {
            const u32x4* xv = reinterpret_cast<const u32x4*>(x + tbase);
            u32x4 r[S];
#pragma unroll
            for (int q = 0; q < S; ++q) r[q] = __builtin_nontemporal_load(xv + q * B + t);
            u32x4* st = reinterpret_cast<u32x4*>(L.tile);
#pragma unroll
            for (int q = 0; q < S; ++q) st[stage_slot<S>(q * B + t)] = r[q];
            __syncthreads();
#pragma unroll
            for (int j = 0; j < S; ++j) {
                const u32x4 a = st[stage_slot<S>(t * S + j)];
                v[4 * j] = a.x;
                v[4 * j + 1] = a.y;
                v[4 * j + 2] = a.z;
                v[4 * j + 3] = a.w;
            }
        }
    }
    if (!staged) {
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
        if (t == 0) {
            L.excl = excl;
            after_lookback();
        }
    }
    __syncthreads();
    const uint32_t pre = L.excl + wpre + (wincl - tot);
    if constexpr (I >= 4) {
        if (staged) {
            // each thread rewrites only the slots it read, then the tile
            // leaves through LDS in lane-consecutive chunks
            u32x4* st = reinterpret_cast<u32x4*>(L.tile);
#pragma unroll
            for (int j = 0; j < S; ++j) {
                u32x4 a;
                a.x = pre + v[4 * j];
                a.y = pre + v[4 * j + 1];
                a.z = pre + v[4 * j + 2];
                a.w = pre + v[4 * j + 3];
                st[stage_slot<S>(t * S + j)] = a;
            }
            __syncthreads();
            u32x4* yv = reinterpret_cast<u32x4*>(y + tbase);
#pragma unroll
            for (int q = 0; q < S; ++q) __builtin_nontemporal_store(st[stage_slot<S>(q * B + t)], yv + q * B + t);
            return;
        }
    }
#pragma unroll
    for (int k = 0; k < I; ++k)
        if (base + k < n) y[base + k] = (int32_t)(pre + v[k]);
}

}  // namespace spmd
