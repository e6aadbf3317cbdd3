// batch.hip -- persistent workgroups draining a device block queue.
//
// Queue layout (all in the caller's workspace):
//   run area    cleared by the prologue kernel on every run:
//                 per segment 1 KiB of fetch cursors (8, 128 B apart),
//                 then per-instance scratch (REDUCE: ticket on its own
//                 line + one status word per block; SCAN: one status
//                 word per tile), 256-byte aligned
//   each area   scratch of the one-launch-per-instance baseline (cleared
//               once at creation; those launches re-arm it themselves)
//   descriptors one 64-byte BatchDesc per instance (immutable)
//   chunk maps  per segment, the instance of every chunk, in queue order
//
// A segment is the work of one persistent kernel: the instances of one
// (class, block size) group at one dependency level.  An instance with no
// dependency is at level 0, one that reads an earlier instance's output is
// one level above it; the levels run one after another, the segments of a
// level side by side.
//
// A chunk is up to `bpf` consecutive logical blocks of one instance; the
// chunks of a segment are numbered instance by instance, blocks ascending,
// so a scan's tiles are fetched in order (its look-back waits only for
// tiles fetched earlier).  A persistent workgroup takes a chunk with one
// relaxed atomic add on a cursor and requests the next chunk as soon as it
// starts the current one, so the atomic's round trip overlaps the block
// bodies (a SCAN worker draws once its tile has published its inclusive
// prefix instead).  A segment cuts its chunks into up to 8 contiguous
// ranges with a cursor each (ChunkRanges below): a range's chunks run on
// one XCD and its draws do not queue behind the other ranges'.  A SCAN
// segment is cut only at instance starts and only when its tiles are small;
// otherwise it keeps one cursor.  A workgroup exits once every cursor it
// draws from has passed the end of its range, so every workgroup ends after
// finitely many fetches.
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <type_traits>
#include <utility>
#include <vector>

#include "cls_hist.hpp"
#include "cls_jacobi.hpp"
#include "cls_reduce.hpp"
#include "cls_scan.hpp"
#include "spmd_batch.h"

namespace spmd {

struct alignas(16) BatchDesc {
    uint32_t cls;
    uint32_t n;        // elements (JACOBI: nx)
    uint32_t ny;       // JACOBI rows
    uint32_t nblocks;  // logical blocks
    uint32_t items;    // items per thread / cells per thread
    uint32_t bpf;      // blocks per fetch
    uint32_t chunk0;   // first chunk of this instance in its group
    uint32_t aux;      // REDUCE/HIST: elements per block; JACOBI: blocks per row
    uint64_t in, out;
    uint64_t ws;       // run-area scratch of this instance
    uint32_t vec;      // in/out 16-byte aligned
    uint32_t pad;
};
static_assert(sizeof(BatchDesc) == 64, "descriptor is 64 bytes");

// One queue per (class, block size): each persistent kernel then holds only
// one class body, which keeps its register use -- and so the number of
// resident workers -- at that class's own level.  Scans of 32 items per
// thread have a queue class of their own, BATCH_SCAN_WIDE (a queue class,
// never a launch's kernel id), so their tiles' registers do not lower the
// occupancy of every scan schedule.  (A 64-item path in the same kernel
// took it to 135 VGPRs, one 512-thread workgroup per CU; 32 items alone
// need 87.)
constexpr int BATCH_SCAN_WIDE = 101;
constexpr int NSIZES = 4, NCLS = 5, NGROUPS = NSIZES * NCLS;
constexpr int NLAUNCH_CLS = 4;  // CLS_ID[0..3] are launch kernel ids
constexpr uint32_t SIZE_B[NSIZES] = {64, 128, 256, 512};
constexpr int CLS_ID[NCLS] = {SPMD_REDUCE_I32, SPMD_SCAN_I32, SPMD_HIST256_U32, SPMD_JACOBI5_F32, BATCH_SCAN_WIDE};
// the launch kernel id whose instances a queue class runs
constexpr int served_by(int cls) { return cls == BATCH_SCAN_WIDE ? SPMD_SCAN_I32 : cls; }
constexpr bool ordered_cls(int cls) { return served_by(cls) == SPMD_SCAN_I32; }

template <int CLS, int B>
struct BatchLdsOf;
template <int B>
struct BatchLdsOf<SPMD_REDUCE_I32, B> {
    ReduceLds<B> r;
};
template <int B>
struct BatchLdsOf<SPMD_SCAN_I32, B> {
    union {
        ScanLds<B, 1> s1;
        ScanLds<B, 2> s2;
        ScanLds<B, 4> s4;
        ScanLds<B, 8> s8;
        ScanLds<B, 16> s16;
    };
};
template <int B>
struct BatchLdsOf<BATCH_SCAN_WIDE, B> {
    ScanLds<B, 32> s32;
};
template <int B>
struct BatchLdsOf<SPMD_HIST256_U32, B> {
    HistLds<HIST_COPIES> h;
};
// the 256-column tile of blocks of 256 or 512 threads; nothing for smaller
// blocks, which run only 64-column blocks
template <int B, int C>
using WideJacobiLds = std::conditional_t<(B >= 256), JacobiWLds<B / 64, C>, char>;

template <int B>
struct BatchLdsOf<SPMD_JACOBI5_F32, B> {
    union {
        JacobiLds<64, B / 64, 1> j1;
        JacobiLds<64, B / 64, 2> j2;
        JacobiLds<64, B / 64, 4> j4;
        JacobiLds<64, B / 64, 8> j8;
        WideJacobiLds<B, 1> w1;  // 256-column groups (blocks of 256 and 512 threads only)
        WideJacobiLds<B, 2> w2;
        WideJacobiLds<B, 4> w4;
    };
};

template <int CLS, int B, typename Hook = NoHook>
__device__ __forceinline__ void run_logical_block(const BatchDesc& d, uint32_t b, BatchLdsOf<CLS, B>& L,
                                                  uint32_t* err, Hook hook = Hook()) {
    const uint32_t t = threadIdx.x;
    if constexpr (CLS == SPMD_REDUCE_I32) {
        uint32_t* ctl = reinterpret_cast<uint32_t*>(d.ws);
        uint64_t* status = reinterpret_cast<uint64_t*>(d.ws + REDUCE_CTL_BYTES);
        reduce_block<B>(reinterpret_cast<const int32_t*>(d.in), nullptr, reinterpret_cast<int32_t*>(d.out), d.n,
                        d.aux, d.nblocks, b, ctl, status, err, d.vec != 0u, L.r);
    } else if constexpr (CLS == SPMD_SCAN_I32) {
        const int32_t* x = reinterpret_cast<const int32_t*>(d.in);
        int32_t* y = reinterpret_cast<int32_t*>(d.out);
        uint64_t* st = reinterpret_cast<uint64_t*>(d.ws);
        const bool v = d.vec != 0u;
        switch (d.items) {
        case 1: scan_tile<B, 1>(x, y, d.n, b, st, 0u, err, v, L.s1, hook); break;
        case 2: scan_tile<B, 2>(x, y, d.n, b, st, 0u, err, v, L.s2, hook); break;
        case 4: scan_tile<B, 4>(x, y, d.n, b, st, 0u, err, v, L.s4, hook); break;
        case 8: scan_tile<B, 8>(x, y, d.n, b, st, 0u, err, v, L.s8, hook); break;
        default: scan_tile<B, 16>(x, y, d.n, b, st, 0u, err, v, L.s16, hook); break;
        }
    } else if constexpr (CLS == BATCH_SCAN_WIDE) {
        const int32_t* x = reinterpret_cast<const int32_t*>(d.in);
        int32_t* y = reinterpret_cast<int32_t*>(d.out);
        uint64_t* st = reinterpret_cast<uint64_t*>(d.ws);
        const bool v = d.vec != 0u;
        scan_tile<B, 32>(x, y, d.n, b, st, 0u, err, v, L.s32, hook);
    } else if constexpr (CLS == SPMD_HIST256_U32) {
        const uint64_t lo = (uint64_t)b * d.aux;
        const uint64_t hi = lo + d.aux < (uint64_t)d.n ? lo + d.aux : (uint64_t)d.n;
        hist_block<B, HIST_COPIES>(reinterpret_cast<const uint32_t*>(d.in), reinterpret_cast<uint32_t*>(d.out), lo,
                                   hi, d.vec != 0u, L.h);
    } else {
        const float* u = reinterpret_cast<const float*>(d.in);
        float* v = reinterpret_cast<float*>(d.out);
        const uint32_t bx = b % d.aux, by = b / d.aux;
        const int tx = (int)(t & 63u), ty = (int)(t >> 6);
        switch (d.items) {
        case 1: jacobi_block<64, B / 64, 1>(u, v, d.n, d.ny, bx, by, tx, ty, L.j1); break;
        case 2: jacobi_block<64, B / 64, 2>(u, v, d.n, d.ny, bx, by, tx, ty, L.j2); break;
        case 4: jacobi_block<64, B / 64, 4>(u, v, d.n, d.ny, bx, by, tx, ty, L.j4); break;
        default: jacobi_block<64, B / 64, 8>(u, v, d.n, d.ny, bx, by, tx, ty, L.j8); break;
        }
    }
}

// JACOBI: the logical blocks of one chunk as a two-stage pipeline -- block
// b+1's global loads are issued before block b's are waited on, so a
// workgroup keeps two tiles' loads in flight.  (Two named register sets,
// not an indexed pair, so nothing goes to scratch.)  Every cell is computed
// as in jacobi_block.
template <int B, int C>
__device__ __forceinline__ void jacobi_chunk(const BatchDesc& d, uint32_t first, uint32_t last,
                                             JacobiLds<64, B / 64, C>& L) {
    constexpr int BY = B / 64;
    const float* u = reinterpret_cast<const float*>(d.in);
    float* v = reinterpret_cast<float*>(d.out);
    const int tx = (int)(threadIdx.x & 63u), ty = (int)(threadIdx.x >> 6);
    const uint32_t w = d.aux;  // blocks per row
    JacobiRegs<64, BY, C> R0, R1;
    jacobi_load<64, BY, C>(u, d.n, d.ny, first % w, first / w, tx, ty, R0);
    for (uint32_t b = first; b < last; b += 2) {
        if (b + 1 < last) jacobi_load<64, BY, C>(u, d.n, d.ny, (b + 1) % w, (b + 1) / w, tx, ty, R1);
        jacobi_commit<64, BY, C>(tx, ty, R0, L);
        __syncthreads();
        jacobi_compute<64, BY, C>(v, d.n, d.ny, b % w, b / w, tx, ty, L);
        __syncthreads();  // the next commit reuses the LDS tile
        if (b + 1 >= last) break;
        if (b + 2 < last) jacobi_load<64, BY, C>(u, d.n, d.ny, (b + 2) % w, (b + 2) / w, tx, ty, R0);
        jacobi_commit<64, BY, C>(tx, ty, R1, L);
        __syncthreads();
        jacobi_compute<64, BY, C>(v, d.n, d.ny, (b + 1) % w, (b + 1) / w, tx, ty, L);
        __syncthreads();
    }
}

// JACOBI, blocks of 256 or 512 threads: inside a chunk, every run of up to
// four 64-column blocks of one row that starts at a multiple of four
// columns-of-blocks and lies wholly in the chunk runs as one 256-column
// tile of the general-width form (jacobi_block_w: each thread four columns
// 64 apart, a wave's loads of a row 1 KiB contiguous); other blocks run one
// by one.  Every cell is computed as in jacobi_block.
template <int B, int C>
__device__ __forceinline__ void jacobi_chunk_grouped(const BatchDesc& d, uint32_t first, uint32_t last,
                                                     JacobiLds<64, B / 64, C>& L64, JacobiWLds<B / 64, C>& LW) {
    constexpr int BY = B / 64;
    const float* u = reinterpret_cast<const float*>(d.in);
    float* v = reinterpret_cast<float*>(d.out);
    const int tx = (int)(threadIdx.x & 63u), ty = (int)(threadIdx.x >> 6);
    const uint32_t w = d.aux;  // 64-column blocks per row
    uint32_t b = first;
    while (b < last) {
        const uint32_t bx = b % w, by = b / w;
        const uint32_t run = min(4u, w - bx);  // blocks of this 256-column group in the row
        if ((bx & 3u) == 0u && b + run <= last) {
            jacobi_block_w<BY, C>(u, v, d.n, d.ny, bx >> 2, by, tx, ty, LW);
            b += run;
        } else {
            jacobi_block<64, BY, C>(u, v, d.n, d.ny, bx, by, tx, ty, L64);
            b += 1;
        }
        __syncthreads();  // the next tile reuses the LDS
    }
}

// REDUCE and HIST: the logical blocks of one fetch cover one contiguous
// element range, so they share one block body -- one LDS sub-histogram
// flushed once, one partial published once -- instead of paying the flush
// or the completion ticket per block.  Integer sums and counts do not
// depend on how the range is cut, so the result is the same.
template <int CLS, int B>
__device__ __forceinline__ void run_fused_chunk(const BatchDesc& d, uint32_t q, uint32_t first, uint32_t last,
                                                BatchLdsOf<CLS, B>& L, uint32_t* err) {
    const uint64_t lo = (uint64_t)first * d.aux;
    const uint64_t end = (uint64_t)last * d.aux;
    const uint64_t hi = end < (uint64_t)d.n ? end : (uint64_t)d.n;
    if constexpr (CLS == SPMD_REDUCE_I32) {
        // chunk q of this instance is block q of a grid of ceil(nblocks / bpf)
        // blocks whose segment is bpf * aux elements (the last one clamped)
        const uint32_t nchunks = (d.nblocks + d.bpf - 1) / d.bpf;
        const uint64_t seg64 = (uint64_t)d.aux * d.bpf;
        const uint32_t seg = seg64 < (uint64_t)d.n ? (uint32_t)seg64 : (d.n ? d.n : 1u);
        uint32_t* ctl = reinterpret_cast<uint32_t*>(d.ws);
        uint64_t* status = reinterpret_cast<uint64_t*>(d.ws + REDUCE_CTL_BYTES);
        reduce_block<B>(reinterpret_cast<const int32_t*>(d.in), nullptr, reinterpret_cast<int32_t*>(d.out), d.n,
                        seg, nchunks, q, ctl, status, err, d.vec != 0u, L.r);
        (void)lo;
        (void)hi;
    } else {
        hist_block<B, HIST_COPIES>(reinterpret_cast<const uint32_t*>(d.in), reinterpret_cast<uint32_t*>(d.out), lo,
                                   hi, d.vec != 0u, L.h);
        (void)q;
        (void)err;
    }
}

// Chunk ranges of a segment.  The chunks are cut into R = min(8, workers)
// contiguous ranges
// with one cursor each, 128 bytes apart.  Worker w belongs to range w mod R:
// the hardware deals a grid's workgroups to the 8 XCDs round-robin, so a
// range runs on one XCD and its instances' lines -- a stencil's neighbouring
// tiles above all -- meet in that XCD's L2, and each cursor takes 1/R of the
// draws.  (Were the dealing different, only the locality would suffer.)
// Range sizes follow the ranges' worker counts, so with as many chunks as
// workers every chunk is some worker's static one.  Worker w's first chunk
// is chunk w div R of its range, taken without a draw; range q's draws hand
// out its chunks from lo(q) + workers(q) on, and a range with no chunk
// beyond the static ones is closed from the start.  Once a range is
// exhausted the worker reads the other open ranges' cursors (one round of
// plain loads, in parallel: a cursor only grows, so a range seen exhausted
// stays so), draws from the next range still open, and exits when none is.
// A SCAN segment's ranges start at instance boundaries and have no static
// chunks: every tile is drawn, so an instance's tiles start in order from
// one cursor and a look-back only waits for tiles that running workers
// already hold (range_table_ordered).
// The host computes the table once per segment; the kernel copies it to
// LDS, where wave 0 reads it at chunk ends.
struct RangeTable {
    uint32_t lo[BATCH_CURSOR_RANGES + 1];   // first chunk of range q; lo[R] = the chunk count
    uint32_t wlo[BATCH_CURSOR_RANGES + 1];  // workers of ranges 0 .. q-1
    uint32_t nrange;                        // R
    uint32_t closed;                        // ranges with no chunk to draw, one bit each
};

// Ranges of a segment whose chunks may run in any order.
RangeTable range_table(uint32_t workers, uint32_t chunks) {
    RangeTable t{};
    const uint32_t R = workers < BATCH_CURSOR_RANGES ? workers : (uint32_t)BATCH_CURSOR_RANGES;
    t.nrange = R;
    for (uint32_t q = 0; q <= R; ++q) {
        t.wlo[q] = R ? q * (workers / R) + (q < workers % R ? q : workers % R) : 0u;
        t.lo[q] = workers ? (uint32_t)((uint64_t)chunks * t.wlo[q] / workers) : 0u;
    }
    for (uint32_t q = 0; q < R; ++q)
        if (t.lo[q + 1] - t.lo[q] <= t.wlo[q + 1] - t.wlo[q]) t.closed |= 1u << q;
    return t;
}

// Ranges of a SCAN segment: cut at the first instance start at or after
// each proportional point (cinst[i] is the instance of chunk i, chunks in
// queue order), all chunks drawn (no static ones).  Only segments of small
// tiles are cut (mean chunk <= SCAN_RANGES_MAX_ELEMS elements), where one
// cursor's serialized draws bound the queue.  Large tiles keep one range:
// measured on the mixed workload's scans, 8 ranges took 4.86 ms against
// 7.11 at 2048-element tiles, were even at 4096 and lost at 8192 (2.79
// against 2.47 ms).
constexpr uint64_t SCAN_RANGES_MAX_ELEMS = 4096;

RangeTable range_table_ordered(uint32_t workers, const std::vector<uint32_t>& cinst, uint64_t elems) {
    RangeTable t{};
    const uint32_t total = (uint32_t)cinst.size();
    const bool cut = total && elems <= SCAN_RANGES_MAX_ELEMS * total;
    const uint32_t R = !cut ? 1u : workers < BATCH_CURSOR_RANGES ? workers : (uint32_t)BATCH_CURSOR_RANGES;
    t.nrange = R;
    uint32_t i = 0;
    for (uint32_t q = 0; q <= R; ++q) {
        const uint32_t target = R ? (uint32_t)((uint64_t)total * q / R) : 0u;
        if (i < target) i = target;
        while (i < total && i > 0 && cinst[i] == cinst[i - 1]) ++i;
        t.lo[q] = q == R ? total : i;
        t.wlo[q] = 0;
    }
    for (uint32_t q = 0; q < R; ++q)
        if (t.lo[q + 1] == t.lo[q]) t.closed |= 1u << q;
    return t;
}

struct ChunkRanges {
    static constexpr uint32_t CURSOR_WORDS = (uint32_t)BATCH_CURSOR_SLOT / 4;
    const RangeTable& T;  // the LDS copy
    uint32_t cur;
    uint32_t done;  // ranges known exhausted, one bit each (wave 0's copy is the live one)
    uint32_t* cursor;

    __device__ ChunkRanges(const RangeTable& t, uint32_t* c)
        : T(t), cur(blockIdx.x % t.nrange), done(t.closed), cursor(c) {}
    __device__ uint32_t total() const { return T.lo[T.nrange]; }
    // chunk of draw value v on range q, or total() if the range has none left
    __device__ uint32_t chunk_of(uint32_t q, uint32_t v) const {
        const uint64_t idx = (uint64_t)T.lo[q] + (T.wlo[q + 1] - T.wlo[q]) + v;
        return idx < (uint64_t)T.lo[q + 1] ? (uint32_t)idx : total();
    }
    // this worker's static chunk, or total() if its range is too short
    __device__ uint32_t first() const {
        const uint32_t c = T.lo[cur] + blockIdx.x / T.nrange;
        return c < T.lo[cur + 1] ? c : total();
    }
    // is there a range to draw from now (false: resolve() without a draw)
    __device__ bool open() const { return !(done >> cur & 1u); }
    // one draw on the current range (one lane)
    __device__ uint32_t draw() const { return atomic_add_dev(cursor + CURSOR_WORDS * cur, 1u); }
    // Wave 0, all 64 lanes: the chunk that lane 0's draw `raw` on the current
    // range gives (when `drawn`), else one from a range still open, else
    // total().  Lane q reads range q's cursor, one ballot marks the exhausted.
    __device__ uint32_t resolve(uint32_t raw, bool drawn) {
        const uint32_t R = T.nrange, all = (1u << R) - 1u, lane = lane64();
        raw = __builtin_amdgcn_readfirstlane(raw);
        for (;;) {
            if (drawn) {
                const uint32_t c = chunk_of(cur, raw);
                if (c < total()) return c;
                done |= 1u << cur;
            }
            if (done == all) return total();
            const uint32_t ql = lane < R ? lane : 0u;  // lanes past R index range 0, unused
            const bool probe = lane < R && !(done >> lane & 1u);
            const uint32_t v = probe ? load_dev(cursor + CURSOR_WORDS * ql) : 0u;
            done |= (uint32_t)__builtin_amdgcn_ballot_w64(probe && chunk_of(ql, v) >= total());
            if (done == all) return total();
            while (done >> cur & 1u) cur = cur + 1u < R ? cur + 1u : 0u;
            raw = 0;
            if (lane == 0) raw = draw();
            raw = __builtin_amdgcn_readfirstlane(raw);
            drawn = true;
        }
    }
};

template <int CLS, int B>
__global__ __launch_bounds__(B) void batch_persistent_kernel(const BatchDesc* __restrict__ descs,
                                                              const uint32_t* __restrict__ chunk_inst,
                                                              uint32_t total_chunks, uint32_t* cursor,
                                                              uint32_t* err, RangeTable ranges) {
    __shared__ BatchLdsOf<CLS, B> L;
    __shared__ uint32_t s_next;
    __shared__ RangeTable s_ranges;
    const uint32_t t = threadIdx.x;
    if (t == 0) s_ranges = ranges;
    __syncthreads();
    ChunkRanges q(s_ranges, cursor);
    constexpr uint32_t SERVED = (uint32_t)served_by(CLS);  // the descriptors' class
    if constexpr (ordered_cls(CLS)) {
        // Every tile is drawn (no static chunks), in order within its range,
        // and a range holds whole instances: a tile is only ever owned by a
        // running worker, so the tiles a look-back waits on are in progress
        // even when other kernels hold some of the compute units.  The next
        // draw is made once the tile has published its inclusive prefix:
        // drawn earlier, a reserved tile that has not started would hold up
        // its successors' look-back while this worker is itself waiting in a
        // look-back.
        if (t < 64) {
            const bool drawn = q.open();
            const uint32_t r = q.resolve(drawn && t == 0 ? q.draw() : 0u, drawn);
            if (t == 0) s_next = r;
        }
        __syncthreads();
        uint32_t c = __builtin_amdgcn_readfirstlane(s_next);
        while (c < total_chunks) {
            __syncthreads();  // every thread has read s_next
            uint32_t raw = 0;
            bool hooked = false;  // thread 0: the look-back hook has run
            const BatchDesc d = descs[chunk_inst[c]];
            const uint32_t first = (c - d.chunk0) * d.bpf;
            const uint32_t last = min(first + d.bpf, d.nblocks);
            if (t == 0 && (first >= last || d.cls != SERVED))
                atomicOr(err, first >= last ? ERRBIT_QUEUE : ERRBIT_BAD_DESC);
            if (d.cls != SERVED) break;
            auto fetch_once = [&]() {  // thread 0, after the tile's look-back
                if (!hooked) {
                    hooked = true;
                    if (q.open()) raw = q.draw();
                }
            };
            for (uint32_t b = first; b < last; ++b) {
                run_logical_block<CLS, B>(d, b, L, err, fetch_once);
                __syncthreads();  // the next logical block reuses the LDS
            }
            if (t < 64) {
                const bool drawn = __builtin_amdgcn_readfirstlane(hooked ? 1u : 0u) != 0u && q.open();
                const uint32_t r = q.resolve(raw, drawn);
                if (t == 0) s_next = r;
            }
            __syncthreads();
            c = __builtin_amdgcn_readfirstlane(s_next);
        }
    } else {
        uint32_t c = __builtin_amdgcn_readfirstlane(q.first());  // block-uniform
        if (c >= total_chunks) {
            if (t < 64) {
                const bool drawn = q.open();
                const uint32_t r = q.resolve(drawn && t == 0 ? q.draw() : 0u, drawn);
                if (t == 0) s_next = r;
            }
            __syncthreads();
            c = __builtin_amdgcn_readfirstlane(s_next);
        }
        while (c < total_chunks) {
            __syncthreads();  // every thread has read s_next
            // the next draw is issued now; its round trip overlaps the chunk
            const bool drawn = t < 64 && q.open();  // wave-uniform in wave 0
            uint32_t raw = 0;
            if (drawn && t == 0) raw = q.draw();
            const BatchDesc d = descs[chunk_inst[c]];
            const uint32_t first = (c - d.chunk0) * d.bpf;
            const uint32_t last = min(first + d.bpf, d.nblocks);
            if (t == 0 && (first >= last || d.cls != SERVED))
                atomicOr(err, first >= last ? ERRBIT_QUEUE : ERRBIT_BAD_DESC);
            if (d.cls != SERVED) break;
            if constexpr (CLS == SPMD_REDUCE_I32 || CLS == SPMD_HIST256_U32) {
                run_fused_chunk<CLS, B>(d, c - d.chunk0, first, last, L, err);
                __syncthreads();
            } else {
                if constexpr (B >= 256) {
                    switch (d.items) {
                    case 1: jacobi_chunk_grouped<B, 1>(d, first, last, L.j1, L.w1); break;
                    case 2: jacobi_chunk_grouped<B, 2>(d, first, last, L.j2, L.w2); break;
                    case 4: jacobi_chunk_grouped<B, 4>(d, first, last, L.j4, L.w4); break;
                    default:
                        for (uint32_t b = first; b < last; ++b) {
                            run_logical_block<CLS, B>(d, b, L, err, NoHook());
                            __syncthreads();  // the next logical block reuses the LDS
                        }
                        break;
                    }
                } else switch (d.items) {
                case 1: jacobi_chunk<B, 1>(d, first, last, L.j1); break;
                case 2: jacobi_chunk<B, 2>(d, first, last, L.j2); break;
                case 4: jacobi_chunk<B, 4>(d, first, last, L.j4); break;
                default:
                    // 8 cells per thread already keep about 10 loads in flight
                    // per thread; a second register set would cost occupancy
                    for (uint32_t b = first; b < last; ++b) {
                        run_logical_block<CLS, B>(d, b, L, err, NoHook());
                        __syncthreads();  // the next logical block reuses the LDS
                    }
                    break;
                }
            }
            if (t < 64) {
                const uint32_t r = q.resolve(raw, drawn);
                if (t == 0) s_next = r;
            }
            __syncthreads();
            c = __builtin_amdgcn_readfirstlane(s_next);
        }
    }
}

// Clears the run area (16-byte words) and the histogram outputs of level 0.
__global__ __launch_bounds__(256) void batch_prologue_kernel(u32x4* run, uint64_t run_words,
                                                             uint32_t* const* hist_out, uint32_t nhist) {
    if (blockIdx.x < nhist) {
        hist_out[blockIdx.x][threadIdx.x] = 0u;
        return;
    }
    const uint64_t stride = (uint64_t)(gridDim.x - nhist) * 256u;
    const u32x4 z = {0u, 0u, 0u, 0u};
    for (uint64_t i = (uint64_t)(blockIdx.x - nhist) * 256u + threadIdx.x; i < run_words; i += stride) run[i] = z;
}

// Clears the histogram outputs of one dependency level above 0, in stream
// order just before that level: an instance of a lower level may still read
// those bins (a histogram's bins are overwritten at its own level, as by a
// run of the instances one by one in level order).
__global__ __launch_bounds__(256) void batch_hist_clear_kernel(uint32_t* const* hist_out) {
    hist_out[blockIdx.x][threadIdx.x] = 0u;
}

}  // namespace spmd

using namespace spmd;

// The instances of one group at one dependency level: one persistent
// kernel per run.
struct BatchSegment {
    uint32_t level;
    int group;
    size_t chunk_off;  // its chunk map in the workspace
    uint32_t chunks;   // chunks in its queue
    uint32_t grid;     // persistent workgroups
    int direct;        // an instance with bpf 0, run as its own grid; -1 for a queue
    RangeTable ranges;  // its chunk ranges (queues only)
};

struct SegKey {
    uint32_t level;
    int group;
    int direct;
    bool operator<(const SegKey& o) const {
        if (level != o.level) return level < o.level;
        if (group != o.group) return group < o.group;
        return direct < o.direct;
    }
    bool operator==(const SegKey& o) const { return level == o.level && group == o.group && direct == o.direct; }
};

struct spmd_batch {
    int n = 0;
    std::vector<spmd_batch_item> items;
    std::vector<spmd_schedule> sched;
    std::vector<uint64_t> blocks;  // logical blocks per instance
    uint8_t* ws = nullptr;
    size_t run_bytes = 0, each_off = 0, desc_off = 0, hist_off = 0;
    std::vector<BatchSegment> seg;  // by level, then group
    // launch order: by level, and within a level the segments with the most
    // estimated work first (segment indices into seg)
    std::vector<uint32_t> order;
    std::vector<size_t> each_ws;        // per instance: offset of its standalone workspace
    std::vector<size_t> each_partials;  // per instance (REDUCE): offset of its partials
    uint32_t nhist = 0;
    // queued HIST outputs in the list at hist_off, by level: level l owns
    // entries [hist_lo[l], hist_lo[l + 1])
    std::vector<uint32_t> hist_lo;
    uint64_t total_blocks = 0, total_chunks = 0;
    uint32_t each_launches = 0;
    const DevInfo* dev = nullptr;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // fork/join of the segment kernels of one level over side streams
    // (levels with two or more segments); per level / per segment, null
    // where unused, all null when the segments run in order
    std::vector<hipEvent_t> ev_fork, ev_join;
};

namespace {

int size_index(uint32_t block) {
    for (int g = 0; g < NSIZES; ++g)
        if (SIZE_B[g] == block) return g;
    return -1;
}
int class_index(int kernel_id) {
    for (int c = 0; c < NLAUNCH_CLS; ++c)
        if (CLS_ID[c] == kernel_id) return c;
    return -1;
}
// queue group of an instance under a schedule: (queue class, block size)
int group_of(int kernel_id, uint32_t block, uint32_t items) {
    const int si = size_index(block);
    int ci = class_index(kernel_id);
    if (kernel_id == SPMD_SCAN_I32 && items >= 32) ci = NLAUNCH_CLS;  // BATCH_SCAN_WIDE
    return (si < 0 || ci < 0) ? -1 : ci * NSIZES + si;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Blocks per fetch actually used.  A SCAN instance fetches one tile per
// chunk: a worker runs the tiles of a chunk one after another, and the
// first tile of the next chunk needs this chunk's last tile's aggregate,
// so chunks of several tiles would run the instance serially.
uint32_t effective_bpf(const spmd_batch_item& it, const spmd_schedule& s) {
    return (it.kernel_id == SPMD_SCAN_I32 || s.bpf == 0) ? 1u : s.bpf;
}

// bpf 0: the instance runs as its class's own grid, outside the queue.
bool is_direct(const spmd_schedule& s) { return s.bpf == 0; }

uint64_t cdiv(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

// Logical blocks of an item under a schedule, 0 if the pair is invalid.
uint64_t item_blocks(const spmd_batch_item& it, const spmd_schedule& s) {
    if (group_of(it.kernel_id, s.block, s.items) < 0) return 0;
    const uint64_t per = (uint64_t)s.block * s.items;
    switch (it.kernel_id) {
    case SPMD_REDUCE_I32:
    case SPMD_SCAN_I32:
    case SPMD_HIST256_U32: {
        const bool wide = it.kernel_id == SPMD_SCAN_I32 && s.items == 32;
        if (s.items != 1 && s.items != 2 && s.items != 4 && s.items != 8 && s.items != 16 && !wide) return 0;
        const uint64_t nb = cdiv(it.n, per);
        return nb ? nb : 1;
    }
    case SPMD_JACOBI5_F32: {
        if (s.items != 1 && s.items != 2 && s.items != 4 && s.items != 8) return 0;
        if (it.n == 0 || it.ny == 0) return 0;
        const uint64_t by = s.block / 64;
        return cdiv(it.n, 64) * cdiv(it.ny, by * s.items);
    }
    default: return 0;
    }
}

}  // namespace

// Does an instance's output overlap its input?  Every class reads its whole
// input before or while it writes, and a batch may run an instance more than
// once (graph replays, the timing of the learned schedule's fallback), so an
// output over the input would be read back as input: SPMD_ERR_ARGS.
namespace spmd {
bool batch_out_overlaps_in(const spmd_batch_item& it) {
    uint64_t in_bytes = 4ull * it.n, out_bytes = 4;
    switch (it.kernel_id) {
    case SPMD_REDUCE_I32: out_bytes = 4; break;
    case SPMD_SCAN_I32: out_bytes = 4ull * it.n; break;
    case SPMD_HIST256_U32: out_bytes = 1024; break;
    case SPMD_JACOBI5_F32: in_bytes = out_bytes = 4ull * it.n * it.ny; break;
    }
    if (!it.in) return false;
    return overlap(it.in, in_bytes, it.out, out_bytes);
}
}  // namespace spmd

namespace {

// Run-area scratch of an instance under the queue.
size_t run_scratch(const spmd_batch_item& it, uint64_t nb) {
    if (it.kernel_id == SPMD_REDUCE_I32) return align_up(REDUCE_CTL_BYTES + 8 * nb, 256);
    if (it.kernel_id == SPMD_SCAN_I32) return align_up(8 * nb, 256);
    return 0;
}

// Scratch of the one-launch baseline (the class's workspace, then REDUCE
// partials), 256-byte aligned pieces.
size_t each_ws_bytes(const spmd_batch_item& it, uint64_t nb) {
    const spmd_dim3 g{(uint32_t)nb, 1, 1}, b{64, 1, 1};
    if (it.kernel_id == SPMD_REDUCE_I32) return align_up(ws_reduce_i32(g, b, it.n), 256);
    if (it.kernel_id == SPMD_SCAN_I32) return align_up(ws_scan_i32(g, b, it.n), 256);
    return 0;
}
size_t each_scratch(const spmd_batch_item& it, uint64_t nb) {
    size_t s = each_ws_bytes(it, nb);
    if (it.kernel_id == SPMD_REDUCE_I32) s += align_up(4 * nb, 256);
    return s;
}

struct Layout {
    size_t cursor_bytes, run_bytes, each_off, each_bytes, desc_off, hist_off, total;
    uint32_t nhist;
    std::vector<uint32_t> level;     // per instance
    std::vector<BatchSegment> seg;   // by level, then group
    std::vector<uint32_t> seg_of;    // per instance: its segment
};

// Estimated device time of a segment: its instances' algorithmic bytes,
// scans weighted 1.5x (a scan's look-back makes it run at about two thirds
// of a streaming class's rate in the queue).  Only the order of segments
// within a level uses it.  On the 10 000-launch mixed workload this puts
// the large-tile scan queue first, then Jacobi: 5.87 ms against 6.1 ms in
// class order; Jacobi first measured 6.55 ms, and splitting the device
// between the first segments in proportion to these costs 7.24 ms (a
// segment then cannot use what the others free when they finish).
double item_cost(const spmd_batch_item& it) {
    switch (it.kernel_id) {
    case SPMD_REDUCE_I32: return 4.0 * it.n;
    case SPMD_SCAN_I32: return 1.5 * 8.0 * it.n;
    case SPMD_HIST256_U32: return 4.0 * it.n;
    case SPMD_JACOBI5_F32: return 8.0 * it.n * it.ny;
    }
    return 0.0;
}

std::vector<double> segment_costs(const spmd_batch_item* items, const Layout& L, int n) {
    std::vector<double> cost(L.seg.size(), 0.0);
    for (int i = 0; i < n; ++i) cost[L.seg_of[i]] += item_cost(items[i]);
    return cost;
}

// Segments of one level run concurrently, but the device runs only a few
// hardware queues at once (4 per process by default), each in submission
// order: the longest segments go first, so none of them waits behind short
// ones and is then left to run alone at the end of the level.
std::vector<uint32_t> launch_order(const std::vector<double>& cost, const Layout& L) {
    const size_t nseg = L.seg.size();
    std::vector<uint32_t> order(nseg);
    for (size_t k = 0; k < nseg; ++k) order[k] = (uint32_t)k;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
        if (L.seg[a].level != L.seg[b].level) return L.seg[a].level < L.seg[b].level;
        return cost[a] > cost[b];
    });
    return order;
}

// Dependency levels: dep[i] is an earlier instance (dep[i] < i) or NO_DEP;
// an instance sits one level above the one it reads.
int dep_levels(const uint32_t* dep, int n, std::vector<uint32_t>& level) {
    level.assign(n, 0);
    if (!dep) return SPMD_OK;
    for (int i = 0; i < n; ++i) {
        if (dep[i] == SPMD_NO_DEP) continue;
        if (dep[i] >= (uint32_t)i) return SPMD_ERR_ARGS;
        level[i] = level[dep[i]] + 1;
    }
    return SPMD_OK;
}

int plan_layout(const spmd_batch_item* items, const spmd_schedule* sched, const uint32_t* dep, int n,
                std::vector<uint64_t>& blocks, Layout& L) {
    if (n <= 0 || !items || !sched) return SPMD_ERR_ARGS;
    blocks.assign(n, 0);
    int rc = dep_levels(dep, n, L.level);
    if (rc) return rc;
    size_t run = 0, each = 0;
    uint32_t nhist = 0;
    std::vector<SegKey> key(n);
    for (int i = 0; i < n; ++i) {
        const auto& it = items[i];
        const auto& s = sched[i];
        if (it.kernel_id != SPMD_REDUCE_I32 && it.kernel_id != SPMD_SCAN_I32 && it.kernel_id != SPMD_HIST256_U32 &&
            it.kernel_id != SPMD_JACOBI5_F32)
            return SPMD_ERR_INVALID_KERNEL;
        const uint64_t nb = item_blocks(it, s);
        if (nb == 0) return SPMD_ERR_INVALID_DIM;
        if (nb >= (1ull << 31)) return SPMD_ERR_INVALID_DIM;
        if (!it.out || (!it.in && it.n)) return SPMD_ERR_ARGS;
        if (batch_out_overlaps_in(it)) return SPMD_ERR_ARGS;
        blocks[i] = nb;
        run += run_scratch(it, nb);
        each += each_scratch(it, nb);
        key[i] = SegKey{L.level[i], group_of(it.kernel_id, s.block, s.items), is_direct(s) ? i : -1};
        if (it.kernel_id == SPMD_HIST256_U32 && !is_direct(s)) ++nhist;
    }
    // segments in (level, group, queue first) order
    std::vector<SegKey> keys(key);
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    L.seg.assign(keys.size(), BatchSegment{});
    std::vector<uint64_t> ch(keys.size(), 0);
    L.seg_of.assign(n, 0);
    for (int i = 0; i < n; ++i) {
        const uint32_t k = (uint32_t)(std::lower_bound(keys.begin(), keys.end(), key[i]) - keys.begin());
        L.seg_of[i] = k;
        if (key[i].direct < 0) ch[k] += cdiv(blocks[i], effective_bpf(items[i], sched[i]));
    }
    L.cursor_bytes = align_up(BATCH_SEG_CURSOR_BYTES * keys.size(), 256);
    L.run_bytes = align_up(L.cursor_bytes + run, 256);
    L.each_off = L.run_bytes;
    L.each_bytes = align_up(each, 256);
    L.desc_off = L.each_off + L.each_bytes;
    L.hist_off = align_up(L.desc_off + sizeof(BatchDesc) * (size_t)n, 256);
    size_t off = align_up(L.hist_off + 8 * (size_t)nhist, 256);
    for (size_t k = 0; k < keys.size(); ++k) {
        if (ch[k] >= (1ull << 31)) return SPMD_ERR_INVALID_DIM;  // chunk numbers + grid fit 32 bits
        BatchSegment& g = L.seg[k];
        g.level = keys[k].level;
        g.group = keys[k].group;
        g.direct = keys[k].direct;
        g.chunk_off = off;
        g.chunks = (uint32_t)ch[k];
        off = align_up(off + 4 * ch[k], 256);
    }
    L.total = off;
    L.nhist = nhist;
    return SPMD_OK;
}

template <int CLS, int B>
int occupancy(int* nb) {
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, batch_persistent_kernel<CLS, B>, B, 0);
    return e == hipSuccess ? SPMD_OK : hip_fail(e);
}

template <int CLS>
int occupancy_b(uint32_t block, int* nb) {
    switch (block) {
    case 64: return occupancy<CLS, 64>(nb);
    case 128: return occupancy<CLS, 128>(nb);
    case 256: return occupancy<CLS, 256>(nb);
    case 512: return occupancy<CLS, 512>(nb);
    }
    return SPMD_ERR_INVALID_DIM;
}

int pool_size(int kernel_id, uint32_t block, uint32_t workers_per_cu, const DevInfo* di, uint32_t* pool) {
    int nb = 0, rc = SPMD_ERR_INVALID_KERNEL;
    switch (kernel_id) {
    case SPMD_REDUCE_I32: rc = occupancy_b<SPMD_REDUCE_I32>(block, &nb); break;
    case SPMD_SCAN_I32: rc = occupancy_b<SPMD_SCAN_I32>(block, &nb); break;
    case BATCH_SCAN_WIDE: rc = occupancy_b<BATCH_SCAN_WIDE>(block, &nb); break;
    case SPMD_HIST256_U32: rc = occupancy_b<SPMD_HIST256_U32>(block, &nb); break;
    case SPMD_JACOBI5_F32: rc = occupancy_b<SPMD_JACOBI5_F32>(block, &nb); break;
    }
    if (rc) return rc;
    if (workers_per_cu && (int)workers_per_cu < nb) nb = (int)workers_per_cu;
    if (nb < 1) nb = 1;
    *pool = (uint32_t)nb * (uint32_t)di->num_cus;
    return SPMD_OK;
}

template <int CLS>
void launch_group(uint32_t block, dim3 gr, hipStream_t s, const BatchDesc* descs, const uint32_t* cmap,
                  uint32_t chunks, uint32_t* cursor, uint32_t* err, const RangeTable& t) {
    switch (block) {
    case 64: hipLaunchKernelGGL((batch_persistent_kernel<CLS, 64>), gr, dim3(64), 0, s, descs, cmap, chunks, cursor, err, t); break;
    case 128: hipLaunchKernelGGL((batch_persistent_kernel<CLS, 128>), gr, dim3(128), 0, s, descs, cmap, chunks, cursor, err, t); break;
    case 256: hipLaunchKernelGGL((batch_persistent_kernel<CLS, 256>), gr, dim3(256), 0, s, descs, cmap, chunks, cursor, err, t); break;
    case 512: hipLaunchKernelGGL((batch_persistent_kernel<CLS, 512>), gr, dim3(512), 0, s, descs, cmap, chunks, cursor, err, t); break;
    }
}

// Side streams for the group kernels, per device, created once with the
// device current and kept for the life of the process (default priority).
// A run forks them from the caller's stream with an event and joins them
// back with one event per group, so runs on one stream stay ordered and a
// captured run becomes a graph with one branch per group.
std::mutex g_side_mu;
hipStream_t g_side[64][NGROUPS];
bool g_side_ready[64];

int side_streams(const DevInfo* di, hipStream_t** out) {
    std::lock_guard<std::mutex> lk(g_side_mu);
    if (di->device < 0 || di->device >= 64) return SPMD_ERR_HIP;
    if (!g_side_ready[di->device]) {
        for (int g = 0; g < NGROUPS; ++g) {
            hipError_t e = hipStreamCreateWithFlags(&g_side[di->device][g], hipStreamNonBlocking);
            if (e != hipSuccess) return hip_fail(e);
        }
        g_side_ready[di->device] = true;
    }
    *out = g_side[di->device];
    return SPMD_OK;
}

// Instance i as its class's own grid (spmd_launch: one logical block per
// workgroup, the hardware dispatcher as the queue), with its scratch in the
// each area.
int launch_direct(spmd_batch* b, int i, hipStream_t stream) {
    const auto& it = b->items[i];
    const auto& s = b->sched[i];
    const uint32_t nb = (uint32_t)b->blocks[i];
    const void* in = it.in;
    void* outp = it.out;
    uint32_t n = it.n, ny = it.ny;
    void* ws = b->ws + b->each_ws[i];
    void* partials = b->ws + b->each_partials[i];
    switch (it.kernel_id) {
    case SPMD_REDUCE_I32: {
        void* args[] = {&in, &partials, &outp, &n, &ws};
        return spmd_launch(SPMD_REDUCE_I32, {nb, 1, 1}, {s.block, 1, 1}, 0, args, stream);
    }
    case SPMD_SCAN_I32: {
        if (n == 0) return SPMD_OK;
        void* args[] = {&in, &outp, &n, &ws};
        return spmd_launch(SPMD_SCAN_I32, {nb, 1, 1}, {s.block, 1, 1}, 0, args, stream);
    }
    case SPMD_HIST256_U32: {
        void* args[] = {&in, &outp, &n};
        return spmd_launch(SPMD_HIST256_U32, {nb, 1, 1}, {s.block, 1, 1}, 0, args, stream);
    }
    case SPMD_JACOBI5_F32: {
        void* args[] = {&in, &outp, &n, &ny};
        const uint32_t gx = (uint32_t)cdiv(n, 64);
        return spmd_launch(SPMD_JACOBI5_F32, {gx, nb / gx, 1}, {64, s.block / 64, 1}, 0, args, stream);
    }
    }
    return SPMD_ERR_INVALID_KERNEL;
}

int launch_segment(const spmd_batch* b, const BatchSegment& g, hipStream_t gs, const BatchDesc* descs,
                   uint32_t* cursor, uint32_t* err) {
    const uint32_t* cmap = reinterpret_cast<const uint32_t*>(b->ws + g.chunk_off);
    const uint32_t block = SIZE_B[g.group % NSIZES];
    const dim3 gr(g.grid);
    switch (CLS_ID[g.group / NSIZES]) {
    case SPMD_REDUCE_I32: launch_group<SPMD_REDUCE_I32>(block, gr, gs, descs, cmap, g.chunks, cursor, err, g.ranges); break;
    case SPMD_SCAN_I32: launch_group<SPMD_SCAN_I32>(block, gr, gs, descs, cmap, g.chunks, cursor, err, g.ranges); break;
    case BATCH_SCAN_WIDE: launch_group<BATCH_SCAN_WIDE>(block, gr, gs, descs, cmap, g.chunks, cursor, err, g.ranges); break;
    case SPMD_HIST256_U32: launch_group<SPMD_HIST256_U32>(block, gr, gs, descs, cmap, g.chunks, cursor, err, g.ranges); break;
    case SPMD_JACOBI5_F32: launch_group<SPMD_JACOBI5_F32>(block, gr, gs, descs, cmap, g.chunks, cursor, err, g.ranges); break;
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? SPMD_OK : hip_fail(e);
}

// Prologue, then the levels in order on `s`; within a level the segments
// fork onto side streams and join back before the next level starts, so a
// level reads what every earlier level wrote (the kernel boundaries make
// those writes visible to all XCDs).
int enqueue_run(spmd_batch* b, hipStream_t s) {
    clear_stale_error();
    const uint64_t run_words = b->run_bytes / 16;
    const uint32_t zero_blocks = (uint32_t)std::min<uint64_t>(1024, std::max<uint64_t>(1, cdiv(run_words, 256)));
    uint32_t* const* hist_list = reinterpret_cast<uint32_t* const*>(b->ws + b->hist_off);
    hipLaunchKernelGGL(batch_prologue_kernel, dim3(b->hist_lo[1] + zero_blocks), dim3(256), 0, s,
                       reinterpret_cast<u32x4*>(b->ws), run_words, hist_list, b->hist_lo[1]);
    const BatchDesc* descs = reinterpret_cast<const BatchDesc*>(b->ws + b->desc_off);
    uint32_t* err = b->dev->err_word;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e);
    hipStream_t* side = nullptr;
    const size_t nseg = b->seg.size();
    for (size_t lo = 0; lo < nseg;) {
        size_t hi = lo;
        while (hi < nseg && b->seg[hi].level == b->seg[lo].level) ++hi;
        const uint32_t lev = b->seg[lo].level;
        if (lev > 0 && b->hist_lo[lev + 1] > b->hist_lo[lev]) {
            hipLaunchKernelGGL(batch_hist_clear_kernel, dim3(b->hist_lo[lev + 1] - b->hist_lo[lev]), dim3(256), 0, s,
                               hist_list + b->hist_lo[lev]);
            if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e);
        }
        const bool fork = hi - lo >= 2 && lev < b->ev_fork.size() && b->ev_fork[lev] != nullptr;
        if (fork) {
            int rc = side ? SPMD_OK : side_streams(b->dev, &side);
            if (rc) return rc;
            if ((e = hipEventRecord(b->ev_fork[lev], s)) != hipSuccess) return hip_fail(e);
        }
        for (size_t pos = lo; pos < hi; ++pos) {
            const size_t k = b->order[pos];  // the level's segments, longest first
            hipStream_t gs = s;
            if (fork) {
                gs = side[pos - lo];
                if ((e = hipStreamWaitEvent(gs, b->ev_fork[lev], 0)) != hipSuccess) return hip_fail(e);
            }
            const BatchSegment& g = b->seg[k];
            int rc = g.direct >= 0 ? launch_direct(b, g.direct, gs)
                                   : launch_segment(b, g, gs, descs, reinterpret_cast<uint32_t*>(b->ws + BATCH_SEG_CURSOR_BYTES * k), err);
            if (rc) return rc;
            if (fork) {
                if ((e = hipEventRecord(b->ev_join[k], gs)) != hipSuccess) return hip_fail(e);
                if ((e = hipStreamWaitEvent(s, b->ev_join[k], 0)) != hipSuccess) return hip_fail(e);
            }
        }
        lo = hi;
    }
    return SPMD_OK;
}

void destroy_events(spmd_batch* b) {
    for (hipEvent_t ev : b->ev_fork)
        if (ev) hipEventDestroy(ev);
    for (hipEvent_t ev : b->ev_join)
        if (ev) hipEventDestroy(ev);
    b->ev_fork.clear();
    b->ev_join.clear();
}

}  // namespace

// For plans destroyed right after one enqueue (spmd_launch_batch): run the
// segment kernels in order on the caller's stream, so no event outlives its
// plan while the GPU still has to reach it.
void spmd::batch_run_in_order(spmd_batch* b) { destroy_events(b); }

extern "C" {

uint64_t spmd_batch_item_blocks(const spmd_batch_item* item, const spmd_schedule* sched) {
    if (!item || !sched) return 0;
    return item_blocks(*item, *sched);
}

size_t spmd_batch_workspace_size_dep(const spmd_batch_item* items, const spmd_schedule* sched, const uint32_t* dep,
                                     int n) {
    std::vector<uint64_t> blocks;
    Layout L;
    if (plan_layout(items, sched, dep, n, blocks, L) != SPMD_OK) return 0;
    return L.total;
}

size_t spmd_batch_workspace_size(const spmd_batch_item* items, const spmd_schedule* sched, int n) {
    return spmd_batch_workspace_size_dep(items, sched, nullptr, n);
}

int spmd_batch_create(const spmd_batch_item* items, const spmd_schedule* sched, int n, void* workspace,
                      size_t ws_bytes, uint32_t workers_per_cu, spmd_batch** out) {
    return spmd_batch_create_dep(items, sched, nullptr, n, workspace, ws_bytes, workers_per_cu, out);
}

int spmd_batch_create_dep(const spmd_batch_item* items, const spmd_schedule* sched, const uint32_t* dep, int n,
                          void* workspace, size_t ws_bytes, uint32_t workers_per_cu, spmd_batch** out) {
    if (!out) return SPMD_ERR_ARGS;
    *out = nullptr;
    std::vector<uint64_t> blocks;
    Layout L;
    int rc = plan_layout(items, sched, dep, n, blocks, L);
    if (rc) return rc;
    if (!workspace || ((uintptr_t)workspace % 256) || ws_bytes < L.total) return SPMD_ERR_WORKSPACE;
    const DevInfo* di = nullptr;
    if ((rc = runtime_dev(&di))) return rc;

    auto* b = new spmd_batch();
    b->n = n;
    b->items.assign(items, items + n);
    b->sched.assign(sched, sched + n);
    b->blocks = blocks;
    b->ws = static_cast<uint8_t*>(workspace);
    b->run_bytes = L.run_bytes;
    b->each_off = L.each_off;
    b->desc_off = L.desc_off;
    b->hist_off = L.hist_off;
    b->nhist = L.nhist;
    b->dev = di;
    b->seg = L.seg;
    const std::vector<double> seg_cost = segment_costs(items, L, n);
    b->order = launch_order(seg_cost, L);

    // descriptors, chunk maps, histogram list, baseline scratch offsets
    const size_t nseg = b->seg.size();
    std::vector<BatchDesc> descs(n);
    std::vector<std::vector<uint32_t>> cmap(nseg);
    for (size_t k = 0; k < nseg; ++k) cmap[k].reserve(b->seg[k].chunks);
    std::vector<std::pair<uint32_t, uint64_t>> hist_lv;  // (level, bins) of queued HIST instances
    size_t run = L.cursor_bytes, each = L.each_off;
    b->each_ws.assign(n, 0);
    b->each_partials.assign(n, 0);
    for (int i = 0; i < n; ++i) {
        const auto& it = items[i];
        const auto& s = sched[i];
        std::vector<uint32_t>& cm = cmap[L.seg_of[i]];
        BatchDesc& d = descs[i];
        memset(&d, 0, sizeof d);
        d.cls = (uint32_t)it.kernel_id;
        d.n = it.n;
        d.ny = it.ny;
        d.nblocks = (uint32_t)blocks[i];
        d.items = s.items;
        d.bpf = effective_bpf(it, s);
        d.chunk0 = (uint32_t)cm.size();
        d.in = (uint64_t)(uintptr_t)it.in;
        d.out = (uint64_t)(uintptr_t)it.out;
        d.ws = (uint64_t)(uintptr_t)(b->ws + run);
        const bool va = ((uintptr_t)it.in % 16) == 0;
        const bool vb = ((uintptr_t)it.out % 16) == 0;
        switch (it.kernel_id) {
        case SPMD_REDUCE_I32:
        case SPMD_HIST256_U32: d.aux = s.block * s.items; d.vec = va; break;
        case SPMD_SCAN_I32: d.vec = va && vb; break;
        case SPMD_JACOBI5_F32: d.aux = (uint32_t)cdiv(it.n, 64); break;
        }
        if (it.kernel_id == SPMD_HIST256_U32 && !is_direct(s))  // own grids clear their bins themselves
            hist_lv.emplace_back(L.level[i], (uint64_t)(uintptr_t)it.out);
        const uint64_t nch = is_direct(s) ? 0 : cdiv(blocks[i], d.bpf);
        for (uint64_t k = 0; k < nch; ++k) cm.push_back((uint32_t)i);
        run += run_scratch(it, blocks[i]);
        if (it.kernel_id == SPMD_REDUCE_I32) {
            b->each_ws[i] = each;
            b->each_partials[i] = each + each_ws_bytes(it, blocks[i]);
        } else if (it.kernel_id == SPMD_SCAN_I32) {
            b->each_ws[i] = each;
        }
        each += each_scratch(it, blocks[i]);
        b->total_blocks += blocks[i];
        b->each_launches += it.kernel_id == SPMD_HIST256_U32 ? 2u : 1u;
    }
    std::stable_sort(hist_lv.begin(), hist_lv.end(),
                     [](const auto& a, const auto& c) { return a.first < c.first; });
    const uint32_t nlev = b->seg.back().level + 1;
    std::vector<uint64_t> hist_ptrs(hist_lv.size());
    b->hist_lo.assign(nlev + 1, 0);
    for (size_t k = 0; k < hist_lv.size(); ++k) {
        hist_ptrs[k] = hist_lv[k].second;
        ++b->hist_lo[hist_lv[k].first + 1];
    }
    for (uint32_t l = 0; l < nlev; ++l) b->hist_lo[l + 1] += b->hist_lo[l];
    hipError_t e = hipMemcpy(b->ws + L.desc_off, descs.data(), sizeof(BatchDesc) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess && !hist_ptrs.empty())
        e = hipMemcpy(b->ws + L.hist_off, hist_ptrs.data(), 8 * hist_ptrs.size(), hipMemcpyHostToDevice);
    for (size_t k = 0; k < nseg && e == hipSuccess; ++k)
        if (!cmap[k].empty())
            e = hipMemcpy(b->ws + b->seg[k].chunk_off, cmap[k].data(), 4 * cmap[k].size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && L.each_bytes) e = hipMemset(b->ws + L.each_off, 0, L.each_bytes);
    if (e != hipSuccess) {
        delete b;
        return hip_fail(e);
    }
    std::vector<uint64_t> seg_elems(nseg, 0);  // elements queued per segment
    for (int i = 0; i < n; ++i) seg_elems[L.seg_of[i]] += items[i].n;
    for (size_t k = 0; k < nseg; ++k) {
        BatchSegment& g = b->seg[k];
        b->total_chunks += g.chunks;
        if (g.direct >= 0) continue;
        uint32_t pool = 0;
        const int cls = CLS_ID[g.group / NSIZES];
        if ((rc = pool_size(cls, SIZE_B[g.group % NSIZES], workers_per_cu, di, &pool))) {
            delete b;
            return rc;
        }
        g.grid = (uint32_t)std::min<uint64_t>(pool, g.chunks);
    }
    for (size_t k = 0; k < nseg; ++k) {
        BatchSegment& g = b->seg[k];
        if (g.direct >= 0) continue;
        const int cls = CLS_ID[g.group / NSIZES];
        g.ranges = ordered_cls(cls) ? range_table_ordered(g.grid, cmap[k], seg_elems[k])
                                    : range_table(g.grid, g.chunks);
    }
    // events for the levels that fork over two or more segments
    const uint32_t nlevels = b->seg.back().level + 1;
    b->ev_fork.assign(nlevels, nullptr);
    b->ev_join.assign(nseg, nullptr);
    e = hipSuccess;
    for (size_t lo = 0; lo < nseg && e == hipSuccess;) {
        size_t hi = lo;
        while (hi < nseg && b->seg[hi].level == b->seg[lo].level) ++hi;
        if (hi - lo >= 2) {
            e = hipEventCreateWithFlags(&b->ev_fork[b->seg[lo].level], hipEventDisableTiming);
            for (size_t k = lo; k < hi && e == hipSuccess; ++k)
                e = hipEventCreateWithFlags(&b->ev_join[k], hipEventDisableTiming);
        }
        lo = hi;
    }
    if (e != hipSuccess) {
        spmd_batch_destroy(b);
        return hip_fail(e);
    }
    *out = b;
    return SPMD_OK;
}

int spmd_batch_launch(spmd_batch* b, void* stream) {
    if (!b) return SPMD_ERR_ARGS;
    return enqueue_run(b, static_cast<hipStream_t>(stream));
}

int spmd_batch_graph_launch(spmd_batch* b, void* stream) {
    if (!b) return SPMD_ERR_ARGS;
    hipError_t e;
    if (!b->exec) {
        if ((e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking)) != hipSuccess) return hip_fail(e);
        if ((e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess) return hip_fail(e);
        int rc = enqueue_run(b, b->cap_stream);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(b->cap_stream, &g);
        if (rc) return rc;
        if (e != hipSuccess) return hip_fail(e);
        b->graph = g;
        if ((e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0)) != hipSuccess) return hip_fail(e);
    }
    e = hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SPMD_OK : hip_fail(e);
}

int spmd_batch_launch_each(spmd_batch* b, void* stream) {
    if (!b) return SPMD_ERR_ARGS;
    for (int i = 0; i < b->n; ++i) {
        const int rc = launch_direct(b, i, static_cast<hipStream_t>(stream));
        if (rc) return rc;
    }
    return SPMD_OK;
}

int spmd_batch_stats(const spmd_batch* b, uint64_t* blocks, uint64_t* chunks, uint32_t* persistent_launches,
                     uint32_t* each_launches) {
    if (!b) return SPMD_ERR_ARGS;
    if (blocks) *blocks = b->total_blocks;
    if (chunks) *chunks = b->total_chunks;
    if (persistent_launches) {
        *persistent_launches = 1u + (uint32_t)b->seg.size();  // prologue + one per segment
    }
    if (each_launches) *each_launches = b->each_launches;
    return SPMD_OK;
}

int spmd_batch_pool_size(int kernel_id, uint32_t block, uint32_t workers_per_cu, uint32_t* pool) {
    if (!pool) return SPMD_ERR_ARGS;
    if (class_index(kernel_id) < 0) return SPMD_ERR_INVALID_KERNEL;
    if (size_index(block) < 0) return SPMD_ERR_INVALID_DIM;
    const DevInfo* di = nullptr;
    int rc = runtime_dev(&di);
    if (rc) return rc;
    return pool_size(kernel_id, block, workers_per_cu, di, pool);
}

int spmd_batch_destroy(spmd_batch* b) {
    if (!b) return SPMD_ERR_ARGS;
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    if (b->cap_stream) hipStreamDestroy(b->cap_stream);
    destroy_events(b);
    delete b;
    return SPMD_OK;
}

}  // extern "C"
