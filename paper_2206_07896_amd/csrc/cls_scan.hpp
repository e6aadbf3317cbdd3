// cls_scan.hpp -- tile body of the SCAN_I32 class (inclusive prefix sum
// modulo 2^32).
//
// A tile is B threads x I items: B*I consecutive elements.
//   1. local scan.  A full, 16-byte aligned tile with I >= 4 is read in
//      rows: wave w owns elements [w*64*I, (w+1)*64*I) of the tile and
//      reads them as I/4 coalesced 1 KiB rows, lane l holding elements
//      4l .. 4l+3 of each row.  Each row is scanned where it lies: the
//      lane's four values, then the 32-lane inclusive scan of the lane
//      totals on each half-wavefront (warp32 DPP scan), the two halves
//      joined by lane 31's total, rows chained by their totals.  Any other
//      tile gives each thread I consecutive items: thread-serial scan, then
//      the 32-lane scan of the thread totals.
//   2. the last lane of each wave (rows) or warp (items) writes its total
//      to LDS; barrier; each thread adds the totals before its own;
//   3. grid carry by decoupled look-back (Merrill and Garland, "Single-pass
//      Parallel Prefix Scan with Decoupled Look-back", 2016): the tile
//      publishes its aggregate, wave 0 reads the status words of up to 64
//      predecessors at a time, sums aggregates back to the nearest inclusive
//      prefix, and publishes its own inclusive prefix; barrier;
//   4. every item gets carry + its in-tile prefix and is stored (rows: as
//      the same coalesced rows).
// Values stay in registers from load to store, and LDS holds only the
// per-wave totals, so residency is set by registers, not by a staging tile.
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

template <int B, int I>
struct ScanLds {
    uint32_t warp[B / 32];  // warp totals (items path) or wave totals (rows path)
    uint32_t excl;
};

// Exclusive carry of `tile`, computed by wave 0 (the 64 lanes call it).
// Every status read is a device-coherent access that leaves the XCD, about
// half a microsecond on gfx950, so the round trips are what a look-back
// costs.  The wave reads a window of LOOKBACK_WINDOW predecessors in one
// round trip (each lane LOOKBACK_PER_LANE words, predecessor
// tile - 1 - (lane + 64 j) in slot j), re-reads with exponential back-off
// only the words that are unpublished and nearer than the nearest inclusive
// prefix, sums the words up to that prefix, and moves back a whole window
// if there is none.  A tile whose predecessor already holds an inclusive
// prefix, or whose unpublished predecessors publish while it waits, is done
// in one round trip plus its waits; one deep in a batch of concurrently
// running tiles finds an inclusive prefix hundreds of tiles back in one
// step instead of one step per 64 tiles.  (Polling the immediate
// predecessor alone before reading the window, which costs a second round
// trip, measured about 1% slower on the 2^26 scan.)
constexpr int LOOKBACK_PER_LANE = 2;
constexpr int LOOKBACK_WINDOW = 64 * LOOKBACK_PER_LANE;

// A tile's aggregate as its status word; tile 0's is its inclusive prefix.
__device__ __forceinline__ void scan_publish_agg(uint64_t* status, uint32_t tile, uint32_t agg, uint32_t tag) {
    status_put(status + tile, status_pack(agg, tile == 0 ? SCAN_INCL : SCAN_AGG, tag));
}

// `published`: the caller has already published the tile's aggregate
// (scan_publish_agg), so only the wait and the inclusive prefix remain.
__device__ __forceinline__ uint32_t scan_lookback(uint64_t* status, uint32_t tile, uint32_t agg, uint32_t tag,
                                                  uint32_t* err, bool published = false) {
    const uint32_t lane = lane64();
    if (tile == 0) {
        if (lane == 0 && !published) status_put(status, status_pack(agg, SCAN_INCL, tag));
        return 0;
    }
    if (lane == 0 && !published) status_put(status + tile, status_pack(agg, SCAN_AGG, tag));
    const uint32_t limit = spin_limit(err);
    uint32_t excl = 0;
    int64_t pos = (int64_t)tile - 1;  // nearest predecessor of this window
    for (;;) {
        uint32_t val[LOOKBACK_PER_LANE], flg[LOOKBACK_PER_LANE];
#pragma unroll
        for (int j = 0; j < LOOKBACK_PER_LANE; ++j) {
            const int64_t idx = pos - (int64_t)lane - 64 * j;
            uint64_t w = 0;
            uint32_t f = SCAN_INCL;  // before tile 0: a zero prefix
            if (idx >= 0) {
                w = status_get(status + idx);
                f = status_flag(w, tag);
            }
            val[j] = (uint32_t)(w >> 32);
            flg[j] = f;
        }
        int jstar = LOOKBACK_PER_LANE;  // slot of the nearest inclusive prefix
        uint32_t kstar = 64;             // its lane
        uint32_t spins = 0, nap = 1;
        for (;;) {
            jstar = LOOKBACK_PER_LANE;
            kstar = 64;
#pragma unroll
            for (int j = LOOKBACK_PER_LANE - 1; j >= 0; --j) {
                const uint64_t inc = __builtin_amdgcn_ballot_w64(flg[j] == SCAN_INCL);
                if (inc) {
                    jstar = j;
                    kstar = (uint32_t)__builtin_ctzll(inc);
                }
            }
            // anything unpublished nearer than the inclusive prefix?
            bool missing = false;
#pragma unroll
            for (int j = 0; j < LOOKBACK_PER_LANE; ++j) {
                const bool nearer = j < jstar || (j == jstar && lane < kstar);
                if (__builtin_amdgcn_ballot_w64(nearer && flg[j] == 0u)) missing = true;
            }
            if (!missing) break;
            if (++spins >= limit) {
                if (lane == 0) atomicOr(err, ERRBIT_SPIN_LIMIT);
#pragma unroll
                for (int j = 0; j < LOOKBACK_PER_LANE; ++j)
                    if (flg[j] == 0u) {
                        val[j] = 0;
                        flg[j] = SCAN_AGG;
                    }
                break;
            }
            backoff_sleep(nap);
            nap = nap < 16u ? nap * 2u : 16u;
#pragma unroll
            for (int j = 0; j < LOOKBACK_PER_LANE; ++j) {
                const int64_t idx = pos - (int64_t)lane - 64 * j;
                if (flg[j] == 0u && idx >= 0) {
                    const uint64_t w = status_get(status + idx);
                    val[j] = (uint32_t)(w >> 32);
                    flg[j] = status_flag(w, tag);
                }
            }
        }
        uint32_t part = 0;
#pragma unroll
        for (int j = 0; j < LOOKBACK_PER_LANE; ++j)
            if (j < jstar || (j == jstar && lane <= kstar)) part += val[j];
        excl += wave_sum(part);
        if (jstar < LOOKBACK_PER_LANE) break;
        pos -= LOOKBACK_WINDOW;
    }
    if (lane == 0) status_put(status + tile, status_pack(excl + agg, SCAN_INCL, tag));
    return excl;
}

struct NoHook {
    __device__ void operator()() const {}
};

// Rows form of a full, 16-byte aligned tile with I >= 4: wave w owns
// elements [w*64*I, (w+1)*64*I) of the tile as I/4 rows of 64 lanes x 4
// consecutive elements.  `wx` / `wy` point at the wave's first element.
template <int I>
__device__ __forceinline__ void scan_rows_load(const int32_t* __restrict__ wx, uint32_t lane, u32x4 (&r)[I / 4]) {
    const u32x4* xv = reinterpret_cast<const u32x4*>(wx);
#pragma unroll
    for (int q = 0; q < I / 4; ++q) r[q] = __builtin_nontemporal_load(xv + q * 64 + lane);
}

// In-wave inclusive scan of the rows in place (each row where it lies: the
// lane's four values, then the 32-lane scan of the lane totals on each
// half-wavefront, the halves joined by lane 31's total, rows chained by
// their totals).  Returns the wave's total (wave-uniform).
template <int I>
__device__ __forceinline__ uint32_t scan_rows_local(uint32_t lane, u32x4 (&r)[I / 4]) {
    uint32_t carry = 0;  // total of the rows before row q
#pragma unroll
    for (int q = 0; q < I / 4; ++q) {
        r[q].y += r[q].x;
        r[q].z += r[q].y;
        r[q].w += r[q].z;
        uint32_t incl = w32_inclusive_add(r[q].w);
        incl += lane >= 32u ? (uint32_t)__builtin_amdgcn_readlane((int)incl, 31) : 0u;
        const uint32_t before = incl - r[q].w + carry;
        r[q].x += before;
        r[q].y += before;
        r[q].z += before;
        r[q].w += before;
        carry += (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
    }
    return carry;
}

template <int I>
__device__ __forceinline__ void scan_rows_store(int32_t* __restrict__ wy, uint32_t lane, const u32x4 (&r)[I / 4],
                                                uint32_t pre) {
    u32x4* yv = reinterpret_cast<u32x4*>(wy);
#pragma unroll
    for (int q = 0; q < I / 4; ++q) {
        u32x4 a = r[q];
        a.x += pre;
        a.y += pre;
        a.z += pre;
        a.w += pre;
        __builtin_nontemporal_store(a, yv + q * 64 + lane);
    }
}

// Block totals of the per-wave (or per-warp) sums in LDS: the tile's
// aggregate and the sum of the slots before `mine`.
template <int NSLOT>
__device__ __forceinline__ void scan_slot_sums(const uint32_t* slot, uint32_t mine, uint32_t& agg, uint32_t& before) {
    agg = 0;
    before = 0;
#pragma unroll
    for (int w = 0; w < NSLOT; ++w) {
        const uint32_t s = slot[w];
        agg += s;
        before += ((uint32_t)w < mine) ? s : 0u;
    }
}

// Items form (partial or unaligned tiles, and I < 4): each thread scans I
// consecutive items, then the 32-lane scan of the thread totals.
template <int B, int I, typename Hook = NoHook>
__device__ __forceinline__ void scan_tile_items(const int32_t* __restrict__ x, int32_t* __restrict__ y, uint32_t n,
                                                uint32_t tile, uint64_t* status, uint32_t tag, uint32_t* err,
                                                ScanLds<B, I>& L, Hook after_lookback = Hook()) {
    constexpr int NW = B / 32;
    const uint32_t t = threadIdx.x;
    const uint64_t base = (uint64_t)tile * ((uint64_t)B * I) + (uint64_t)t * I;
    if constexpr (I > 64) {
        // Two rolled passes (the thread's total, then after the look-back
        // the running prefix, re-reading x), so this path neither grows the
        // registers nor unrolls into the code of the rows loop it shares a
        // kernel with: fully unrolled at 128 items it made that kernel
        // three times larger and its full tiles 3% slower.
        uint32_t tot = 0;
#pragma unroll 4
        for (int k = 0; k < I; ++k) tot += (base + k < n) ? (uint32_t)x[base + k] : 0u;
        const uint32_t wincl = w32_inclusive_add(tot);
        if ((t & 31u) == 31u) L.warp[t >> 5] = wincl;
        __syncthreads();
        uint32_t agg, wpre;
        scan_slot_sums<NW>(L.warp, t >> 5, agg, wpre);
        if (t < 64) {
            const uint32_t excl = scan_lookback(status, tile, agg, tag, err);
            if (t == 0) {
                L.excl = excl;
                after_lookback();
            }
        }
        __syncthreads();
        uint32_t run = L.excl + wpre + (wincl - tot);
#pragma unroll 4
        for (int k = 0; k < I; ++k)
            if (base + k < n) {
                run += (uint32_t)x[base + k];
                y[base + k] = (int32_t)run;
            }
        return;
    }
    uint32_t v[I];
#pragma unroll
    for (int k = 0; k < I; ++k) v[k] = (base + k < n) ? (uint32_t)x[base + k] : 0u;
#pragma unroll
    for (int k = 1; k < I; ++k) v[k] += v[k - 1];
    const uint32_t tot = v[I - 1];
    const uint32_t wincl = w32_inclusive_add(tot);
    if ((t & 31u) == 31u) L.warp[t >> 5] = wincl;
    __syncthreads();
    uint32_t agg, wpre;
    scan_slot_sums<NW>(L.warp, t >> 5, agg, wpre);
    if (t < 64) {
        const uint32_t excl = scan_lookback(status, tile, agg, tag, err);
        if (t == 0) {
            L.excl = excl;
            after_lookback();
        }
    }
    __syncthreads();
    const uint32_t pre = L.excl + wpre + (wincl - tot);
#pragma unroll
    for (int k = 0; k < I; ++k)
        if (base + k < n) y[base + k] = (int32_t)(pre + v[k]);
}

// Scan tile `tile` of x into y.  Thread 0 calls `after_lookback` once the
// tile's inclusive prefix is published, i.e. once no other tile can wait on
// this one any more.  Every thread's last access to L comes after the
// tile's second (last) barrier and is a read of L.excl, and a tile writes L
// only before its first barrier (L.warp) or by thread 0 between the two
// (L.excl): back-to-back scan tiles need no barrier between them, a caller
// that puts anything else in the area places one first.
template <int B, int I, typename Hook = NoHook>
__device__ __forceinline__ void scan_tile(const int32_t* __restrict__ x, int32_t* __restrict__ y, uint32_t n,
                                          uint32_t tile, uint64_t* status, uint32_t tag, uint32_t* err, bool vec,
                                          ScanLds<B, I>& L, Hook after_lookback = Hook()) {
    constexpr uint64_t T = (uint64_t)B * I;
    const uint32_t t = threadIdx.x;
    const uint64_t tbase = (uint64_t)tile * T;
    if constexpr (I >= 4) {
        if (vec && tbase + T <= (uint64_t)n) {
            const uint32_t lane = lane64(), wave = t >> 6;
            const uint64_t wbase = tbase + (uint64_t)wave * 64u * I;
            u32x4 r[I / 4];
            scan_rows_load<I>(x + wbase, lane, r);
            const uint32_t carry = scan_rows_local<I>(lane, r);
            if (lane == 0) L.warp[wave] = carry;
            __syncthreads();
            uint32_t agg, wpre;
            scan_slot_sums<B / 64>(L.warp, wave, agg, wpre);
            if (t < 64) {
                const uint32_t excl = scan_lookback(status, tile, agg, tag, err);
                if (t == 0) {
                    L.excl = excl;
                    after_lookback();
                }
            }
            __syncthreads();
            scan_rows_store<I>(y + wbase, lane, r, L.excl + wpre);
            return;
        }
    }
    scan_tile_items<B, I>(x, y, n, tile, status, tag, err, L, after_lookback);
}

}  // namespace spmd
