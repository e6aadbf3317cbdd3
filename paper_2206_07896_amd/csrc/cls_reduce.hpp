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
    uint32_t epoch;
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

// Thread t's share of x[lo, hi): the segment is walked in rows of B
// 16-byte chunks (one per thread), four rows in flight per step, starting
// at a row that depends on the block: blocks whose segments lie a large
// power of two apart then do not stream the same memory channels in
// lockstep.  Integer sums do not depend on the order.
template <int B>
__device__ __forceinline__ uint32_t segment_sum(const int32_t* __restrict__ x, uint64_t lo, uint64_t hi, bool vec,
                                                uint32_t bid) {
    const uint32_t t = threadIdx.x;
    uint32_t acc = 0;
    if (lo >= hi) return 0;
    if (vec) {
        const u32x4* xv = reinterpret_cast<const u32x4*>(x + lo);
        const uint64_t nv = (hi - lo) >> 2;
        const uint64_t rows = nv / B;  // full rows
        const uint64_t r0 = rows ? (bid * 7u) % rows : 0;
        uint64_t r = 0;
        for (; r + 4 <= rows; r += 4) {
            u32x4 a[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                uint64_t row = r0 + r + q;
                row = row >= rows ? row - rows : row;
                a[q] = __builtin_nontemporal_load(xv + row * B + t);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) acc += (a[q].x + a[q].y) + (a[q].z + a[q].w);
        }
        for (; r < rows; ++r) {
            uint64_t row = r0 + r;
            row = row >= rows ? row - rows : row;
            const u32x4 a = __builtin_nontemporal_load(xv + row * B + t);
            acc += (a.x + a.y) + (a.z + a.w);
        }
        for (uint64_t k = rows * B + t; k < nv; k += B) {
            const u32x4 a = __builtin_nontemporal_load(xv + k);
            acc += (a.x + a.y) + (a.z + a.w);
        }
        for (uint64_t j = lo + (nv << 2) + t; j < hi; j += B) acc += (uint32_t)x[j];
    } else {
        for (uint64_t j = lo + t; j < hi; j += B) acc += (uint32_t)x[j];
    }
    return acc;
}

constexpr uint32_t REDUCE_SUBTICKETS = 64;   // first-level ticket counters
constexpr uint32_t REDUCE_TICKET_STRIDE = 32;  // u32 words between counters (128 B)
constexpr size_t REDUCE_CTL_BYTES = (REDUCE_SUBTICKETS + 1) * REDUCE_TICKET_STRIDE * 4;
// The launch epoch: in the top counter's line, 64 bytes past the counter.
// It tags the launch's status words, and the finishing block advances it.
constexpr uint32_t REDUCE_EPOCH_WORD = 16;

// Two-level completion ticket.  Counters on one address serialise at the
// device coherence point, so block b counts on sub-counter b % 64 (each on
// its own cache line); the block completing a sub-counter's group counts
// once on the top counter, and the block completing the top counter is the
// last of the grid.  Each completing block re-arms the counter it completed.
__device__ __forceinline__ bool reduce_ticket_last(uint32_t* ctl, uint32_t G, uint32_t bid) {
    const uint32_t sub = bid % REDUCE_SUBTICKETS;
    const uint32_t members = (G - sub + REDUCE_SUBTICKETS - 1) / REDUCE_SUBTICKETS;
    uint32_t* c1 = ctl + (1 + sub) * REDUCE_TICKET_STRIDE;
    if (atomic_add_dev(c1, 1u) != members - 1u) return false;
    put_dev(c1, 0u);
    const uint32_t groups = G < REDUCE_SUBTICKETS ? G : REDUCE_SUBTICKETS;
    if (atomic_add_dev(ctl, 1u) != groups - 1u) return false;
    put_dev(ctl, 0u);
    return true;
}

// The finishing block: sum the `count` status words (eight independent
// loads in flight per thread; only words not yet visible are polled
// again), write *out and advance the epoch, so words of this launch -- even
// one stored late, after a wait gave up -- read as unwritten in the next.
template <int B>
__device__ __forceinline__ void reduce_final(uint64_t* status, uint32_t count, uint32_t tag, uint32_t* ctl,
                                             int32_t* out, uint32_t* err, ReduceLds<B>& L) {
    const uint32_t limit = spin_limit(err);
    uint32_t acc = 0;
    for (uint32_t j0 = threadIdx.x; j0 < count; j0 += 8u * B) {
        uint64_t w[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const uint32_t j = j0 + (uint32_t)q * B;
            w[q] = j < count ? status_get(status + j) : status_pack(0u, 1u, tag);
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const uint32_t j = j0 + (uint32_t)q * B;
            for (uint32_t spins = 0; status_flag(w[q], tag) == 0u; ++spins) {
                if (spins >= limit) {
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
    if (threadIdx.x == 0) {
        *out = (int32_t)total;
        put_dev(ctl + REDUCE_EPOCH_WORD, tag + 1u);  // every block of this launch has read the epoch
    }
}

// One logical block `bid` of a G-block reduction.  Cross-block state
// (`ctl`, `status`): `ctl` holds the two-level completion ticket and the
// launch epoch (REDUCE_CTL_BYTES), status[b] the partial of block b as a
// status word tagged with the epoch.  Thread 0 publishes the block's
// partial (to `partials`, when given, and as a status word), then takes a
// ticket; the last block reads the G status words (waiting, boundedly, for
// any not yet visible), sums them, writes *out and advances the epoch, so
// words of this launch -- even one stored late, after a wait gave up --
// read as unwritten in the next.  Returns true in the block that finished.
template <int B>
__device__ __forceinline__ bool reduce_block(const int32_t* __restrict__ x, int32_t* partials, int32_t* out,
                                             uint32_t n, uint32_t seg, uint32_t G, uint32_t bid, uint32_t* ctl,
                                             uint64_t* status, uint32_t* err, bool vec, ReduceLds<B>& L) {
    const uint64_t lo = (uint64_t)bid * seg;
    const uint64_t hi = lo + seg < (uint64_t)n ? lo + seg : (uint64_t)n;
    // the epoch's round trip overlaps the segment's loads
    const uint32_t epoch = threadIdx.x == 0 ? load_dev(ctl + REDUCE_EPOCH_WORD) : 0u;
    const uint32_t tot = block_sum_t0<B>(segment_sum<B>(x, lo, hi, vec, bid), L);
    if (threadIdx.x == 0) {
        if (partials) partials[bid] = (int32_t)tot;
        status_put(status + bid, status_pack(tot, 1u, epoch));
        L.last = reduce_ticket_last(ctl, G, bid) ? 1u : 0u;
        L.epoch = epoch;
    }
    __syncthreads();
    const bool last = L.last != 0u;
    const uint32_t tag = L.epoch;
    __syncthreads();
    if (!last) return false;
    reduce_final<B>(status, G, tag, ctl, out, err, L);
    return true;
}


// K consecutive logical blocks [K w, K w + K) of a G-block reduction run by
// workgroup w of P (the launcher's persistent form: P covers the device's
// resident workgroups, so fewer workgroups than logical blocks each keep
// more loads in flight).  Each logical block's sum is computed and written
// to `partials` exactly as a block of its own would; one status word and
// one completion ticket per workgroup carry the workgroup's total, and the
// finishing workgroup sums the P totals.
template <int B, int K>
__device__ __forceinline__ void reduce_blocks(const int32_t* __restrict__ x, int32_t* partials, int32_t* out,
                                              uint32_t n, uint32_t seg, uint32_t G, uint32_t P, uint32_t w,
                                              uint32_t* ctl, uint64_t* status, uint32_t* err, bool vec,
                                              ReduceLds<B>& L, uint32_t (&wsum)[K][B / 64]) {
    const uint32_t t = threadIdx.x;
    const uint32_t b0 = w * K;
    const uint32_t epoch = t == 0 ? load_dev(ctl + REDUCE_EPOCH_WORD) : 0u;
    uint32_t acc[K];
    uint64_t lo[K], hi[K], nv[K];
    uint64_t nvmax = 0;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        acc[j] = 0;
        lo[j] = (uint64_t)(b0 + j) * seg;
        hi[j] = b0 + j < G ? (lo[j] + seg < (uint64_t)n ? lo[j] + seg : (uint64_t)n) : lo[j];
        if (hi[j] < lo[j]) hi[j] = lo[j];
        nv[j] = vec ? (hi[j] - lo[j]) >> 2 : 0;  // whole 16-byte groups (seg is a multiple of 4)
        nvmax = nv[j] > nvmax ? nv[j] : nvmax;
    }
    // the K segments' 16-byte groups, four rows of B per segment in flight
    const u32x4* xv = reinterpret_cast<const u32x4*>(x);
    for (uint64_t v0 = t; v0 < nvmax; v0 += 4u * B) {
        u32x4 a[K][4];
#pragma unroll
        for (int j = 0; j < K; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint64_t v = v0 + (uint64_t)q * B;
                a[j][q] = v < nv[j] ? __builtin_nontemporal_load(xv + (lo[j] >> 2) + v) : u32x4{0u, 0u, 0u, 0u};
            }
#pragma unroll
        for (int j = 0; j < K; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[j] += (a[j][q].x + a[j][q].y) + (a[j][q].z + a[j][q].w);
    }
    // what is left: the last segment's tail, or everything when unaligned
#pragma unroll
    for (int j = 0; j < K; ++j)
        for (uint64_t e = lo[j] + (nv[j] << 2) + t; e < hi[j]; e += B) acc[j] += (uint32_t)x[e];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const uint32_t s = wave_sum(acc[j]);
        if (lane64() == 0) wsum[j][t / 64] = s;
    }
    __syncthreads();
    if (t == 0) {
        uint32_t total = 0;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            uint32_t s = 0;
#pragma unroll
            for (int i = 0; i < B / 64; ++i) s += wsum[j][i];
            if (b0 + j < G) {
                if (partials) partials[b0 + j] = (int32_t)s;
                total += s;
            }
        }
        status_put(status + w, status_pack(total, 1u, epoch));
        L.last = reduce_ticket_last(ctl, P, w) ? 1u : 0u;
        L.epoch = epoch;
    }
    __syncthreads();
    const bool last = L.last != 0u;
    const uint32_t tag = L.epoch;
    __syncthreads();
    if (last) reduce_final<B>(status, P, tag, ctl, out, err, L);
}

}  // namespace spmd
