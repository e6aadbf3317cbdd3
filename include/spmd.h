/* spmd.h -- C ABI of the MI355X (gfx950) SPMD kernel-grid executor.
 *
 * The library runs a fixed set of SPMD kernel classes, written by hand in HIP
 * for gfx950, with the launch semantics of a CUDA grid: thread blocks whose
 * threads run in phases separated by barriers, per-block shared memory (LDS),
 * 32-lane warp shuffle/vote operations (kept on half-wavefronts of the
 * 64-lane hardware wave) and atomics.  Blocks are dispatched either one grid
 * per launch (the hardware dispatcher hands out workgroups) or, for a batch
 * of many launches, by persistent workgroups that fetch chunks of logical
 * blocks from a device queue -- the GPU form of the paper's task queue with
 * coarse-grained fetching (Section IV, Section IV-A).
 *
 * Conventions (all entry points):
 *  - Every function is extern "C", takes plain pointers and sizes, and
 *    returns an int status: SPMD_OK (0) or a negative SPMD_ERR_* code.
 *    Validation errors are returned before anything is enqueued and leave no
 *    state behind.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Launches are asynchronous with respect to the host, as in the paper's
 *    runtime where the host continues after pushing a task (Section IV,
 *    "Push task queue"); a host read of a result needs spmd_sync first (the
 *    barrier the paper inserts between a launch and a dependent copy,
 *    Section III-C1).
 *  - Kernel arguments are packed the way the paper's host prologue packs
 *    them (Section III-C2): `args[i]` points to the value of parameter i (a
 *    device pointer variable for pointer parameters, a uint32_t for sizes).
 *    The values are read and copied during the call; `args` and what it
 *    points to may be reused as soon as the call returns.
 *  - Every data pointer is a device pointer owned by the caller, which keeps
 *    it alive until the work completes.  Scratch memory ("workspace") is
 *    also the caller's: it is sized by spmd_workspace_size, must be
 *    zero-filled once before its first use, and is left reusable by every
 *    launch that completes.  Two launches in flight at the same time must
 *    not share a workspace.
 *  - The library owns only immutable state (dispatch tables, device
 *    attributes) and one device error word per device, which kernels set on
 *    an internal failure and spmd_sync reports and clears.
 */
#ifndef SPMD_H
#define SPMD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    uint32_t x, y, z;
} spmd_dim3;

/* ------------------------------------------------------------------------
 * Status codes
 * ---------------------------------------------------------------------- */
enum {
    SPMD_OK = 0,
    SPMD_ERR_INVALID_KERNEL = -1, /* unknown kernel id                                   */
    SPMD_ERR_INVALID_DIM = -2,    /* zero dimension, block product > 1024, grid product
                                     >= 2^32, or a shape the class does not accept      */
    SPMD_ERR_SHMEM = -3,          /* dynamic + static shared memory over the device or
                                     class limit, or below what the class needs          */
    SPMD_ERR_ARGS = -4,           /* null args / null pointer / size mismatch            */
    SPMD_ERR_HIP = -5,            /* a HIP runtime call failed                           */
    SPMD_ERR_DEVICE = -6,         /* a kernel set the device error word                  */
    SPMD_ERR_TIMEOUT = -7,        /* spmd_sync_timeout ran out of time                   */
    SPMD_ERR_WORKSPACE = -8       /* workspace missing, too small or misaligned          */
};

/* ------------------------------------------------------------------------
 * Kernel classes.  For each: parameters (the order of args[]), launch-shape
 * rules, and what is computed.  Integer classes compute in uint32 arithmetic
 * (sums wrap modulo 2^32 and are returned as int32 bit patterns).
 * ---------------------------------------------------------------------- */
enum {
    /* Block tree reduction, one partial per block, then the last block to
     * finish sums the partials.
     * args: const int32_t* x, int32_t* partials, int32_t* out, uint32_t n,
     *       void* workspace (spmd_workspace_size bytes = 8320 + 8G, 16-byte
     *       aligned)
     * grid (G,1,1), block (B,1,1) with B a power of two in [64, 1024].
     * Block b owns x[b*S, min((b+1)*S, n)), S = 4*ceil(n / (4G))
     * (SPMD_ERR_INVALID_DIM when S does not fit 32 bits: G = 1 and
     * n > 2^32 - 4); partials[b] = sum of its elements, *out = sum of all n
     * elements. */
    SPMD_REDUCE_I32 = 1,

    /* Inclusive prefix sum: y[i] = x[0] + ... + x[i] (mod 2^32), single
     * pass with decoupled look-back across tiles.
     * args: const int32_t* x, int32_t* y, uint32_t n, void* workspace
     * grid (G,1,1), block (B,1,1), B in {64,128,256,512,1024}.  Block g
     * (in the order blocks start) scans a tile of B*I consecutive elements,
     * I = the smallest power of two >= ceil(n / (G*B)); I <= 32 (I <= 128 for B <= 512).
     * x and y may not overlap (SPMD_ERR_ARGS). */
    SPMD_SCAN_I32 = 2,

    /* 256-bin histogram of keys & 255 with per-block LDS sub-histograms
     * (LDS atomics) flushed to hist with global atomics.  hist is
     * overwritten: the library clears it in stream order before counting.
     * args: const uint32_t* keys, uint32_t* hist, uint32_t n
     * grid (G,1,1), block (B,1,1), B a power of two in [64, 1024].  Block b
     * counts keys[b*S, min((b+1)*S, n)), S = 4*ceil(n / (4G))
     * (SPMD_ERR_INVALID_DIM when S does not fit 32 bits: G = 1 and
     * n > 2^32 - 4). */
    SPMD_HIST256_U32 = 3,

    /* One sweep of the 5-point Laplace-Jacobi stencil on an ny x nx
     * row-major fp32 grid: interior u'[i][j] = 0.25f*((u[i-1][j] +
     * u[i+1][j]) + (u[i][j-1] + u[i][j+1])), each operation rounded to
     * fp32 in that order; border cells copied.  Each block stages its tile
     * and a one-cell halo in LDS, barrier, then computes.
     * args: const float* u, float* u_next, uint32_t nx, uint32_t ny
     * block (BX,BY,1) with (BX,BY) in {(16,16), (32,8), (64,1), (64,2),
     * (64,4), (64,8), (128,2), (128,4), (256,1)}; grid (GX,GY,1) with GX*BX >= nx; each
     * thread computes C cells down its column, C = the smallest power of
     * two >= ceil(ny / (GY*BY)), C <= 16.  u and u_next may not overlap. */
    SPMD_JACOBI5_F32 = 4,

    /* C = A * B, fp32 row-major, fp32 accumulation on the matrix cores
     * (v_mfma_f32_32x32x2f32), LDS-staged T x T output tiles.
     * args: const float* A, const float* B, float* C, uint32_t M,
     *       uint32_t N, uint32_t K
     * block (256,1,1); grid (GX,GY,1); the tile edge T is the smallest of
     * {64, 128, 256} with GX*T >= N and GY*T >= M (at 256 each wave holds
     * a 128 x 128 block of C in accumulator registers, one wave per SIMD). */
    SPMD_GEMM_F32 = 5,

    /* Conformance of the 32-lane warp operations on half-wavefronts.
     * args: const int32_t* val, const uint32_t* pred, int32_t* out
     * grid (G,1,1), block (B,1,1), B a multiple of 32.  With T = G*B
     * threads and case c in [0, SPMD_WARPTEST_NCASES):
     *   out[c*T + t] = result of case c on thread t, where
     *   c <  768: op = (shfl, shfl_up, shfl_down, shfl_xor)[c / 192],
     *             width = 1 << ((c / 32) % 6), parameter = c % 32,
     *             applied to val (runtime parameter);
     *   c <  864: vote = (ballot, any, all)[(c - 768) / 32] over predicate
     *             bit (c - 768) % 32 of pred;
     *   c <  904: k = c - 864, op = (up, down, xor, shfl)[k / 10],
     *             width = 32 >> ((k / 5) % 2), parameter 1 << (k % 5), with
     *             parameter and width known at compile time.
     * Semantics follow CUDA's documented shfl/vote behaviour for full
     * masks: a lane reading outside its width segment keeps its own value
     * (xor may read earlier segments). */
    SPMD_WARPTEST = 6,

    /* The paper's dynamic-shared-memory example (Section III, listing
     * cuda_reverse): one block of n threads, s[t] = d[t]; barrier;
     * d[t] = s[n-1-t].
     * args: int32_t* d, uint32_t n
     * grid (1,1,1), block (n,1,1), dyn_shmem >= 4*n. */
    SPMD_REVERSE_I32 = 7,

    /* Stream compaction, a database selection (the filter operators of the
     * GPU database queries covered in Section V-A): y[0, m) = the elements
     * of x strictly greater than t (t is the int32 whose bits the uint32
     * argument holds), in input order, and *count = m.  Elements of y from
     * m on are untouched.  Each 32-lane warp finds its elements' output
     * offsets by ballot and popc; tiles are chained by decoupled look-back
     * over their counts, in ticket order, as SPMD_SCAN_I32.
     * args: const int32_t* x, int32_t* y, uint32_t* count, uint32_t n,
     *       uint32_t t, void* workspace
     * grid (G,1,1), block (B,1,1), B a power of two in [64, 1024]; each
     * thread handles I items, I = the smallest power of two >=
     * ceil(n / (G*B)), I <= 32 (I <= 64 for B <= 512).  workspace:
     * spmd_workspace_size() bytes,
     * 16-byte aligned, zero-filled before first use, then reusable as for
     * SCAN.  y must hold n elements; x may overlap neither y nor count
     * (SPMD_ERR_ARGS). */
    SPMD_COMPACT_I32 = 8,

    /* S fused sweeps of the SPMD_JACOBI5_F32 stencil in one pass over HBM
     * (temporal blocking; the roofline discussion of Section VI-B: a
     * one-sweep stencil is bound by memory, so more sweeps per byte moved
     * is the way past that bound).  u_next = S sweeps of u, every cell
     * computed exactly as by S one-sweep launches (bit-identical).  Each
     * workgroup holds a 256-column region -- a (256 - 2H) x 64 interior
     * tile plus a halo of H = 4 cells (S <= 4) or H = 8 cells (S <= 8) --
     * in registers, sweeps there, and stores the interior.
     * args: const float* u, float* u_next, uint32_t nx, uint32_t ny,
     *       uint32_t sweeps (S, 1..8)
     * block (256,1,1); grid (GX,GY,1) with GX*(256 - 2H) >= nx and
     * GY*64 >= ny.
     * nx must be a multiple of 4, u and u_next 16-byte aligned and not
     * overlapping (SPMD_ERR_ARGS otherwise). */
    SPMD_JACOBI5T_F32 = 9
};

#define SPMD_NUM_KERNELS 9
#define SPMD_WARPTEST_NCASES 904

/* Launch one grid of kernel class `kernel_id` on `stream` (Section IV, "Push
 * task queue": the launch records grid, block, dynamic shared memory and the
 * packed arguments and returns without waiting).  `dyn_shmem` bytes of
 * dynamic LDS are reserved per block in addition to the class's static LDS.
 * Returns SPMD_OK once the work is enqueued. */
int spmd_launch(int kernel_id, spmd_dim3 grid, spmd_dim3 block, size_t dyn_shmem, void** args, void* stream);

/* spmd_launch with its kernels' device time: Section V's roofline places a
 * kernel by its execution time alone, without the host or the stream
 * around it.  `start_event` and `stop_event` are hipEvent_t handles created
 * with timing enabled and owned by the caller; `stop_event` must not be
 * null (SPMD_ERR_ARGS).  The start event is bound to the launch's first
 * kernel dispatch and the stop event to its last, so
 * hipEventElapsedTime(start, stop) is the time from the first kernel's start
 * to the last kernel's end, with no marker packet of hipEventRecord's on
 * the stream.  A null `start_event` binds the stop event alone, which costs
 * the stream nothing (a bound start event costs about as much as a
 * marker): the span is then taken from an earlier event, such as the stop
 * event of the launch before, and also holds the gap between the two
 * launches.  A launch that enqueues no kernel (n = 0) records its events on
 * `stream` together.  Otherwise as spmd_launch, with the same errors; on an
 * error no event is recorded. */
int spmd_launch_timed(int kernel_id, spmd_dim3 grid, spmd_dim3 block, size_t dyn_shmem, void** args, void* stream,
                      void* start_event, void* stop_event);

/* spmd_launch for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same classes, shapes, semantics and errors as spmd_launch, except that
 * the classes with a workspace (SPMD_REDUCE_I32, SPMD_SCAN_I32,
 * SPMD_COMPACT_I32) take args WITHOUT their last parameter, the workspace:
 * the launch uses instead a region of a static device array that the
 * library holds on every device it runs on (SPMD_NOALLOC_REGION_BYTES per
 * class, about 3 MiB per device in all, held until the process ends).
 * Other classes are launched exactly as by spmd_launch.
 *  - Limit: a grid whose workspace (spmd_workspace_size) exceeds
 *    SPMD_NOALLOC_REGION_BYTES -- more than 2^17 blocks -- returns
 *    SPMD_ERR_WORKSPACE before anything is enqueued.
 *  - Allocation: none.  The call makes no hipMalloc/hipFree and calls no
 *    allocating routine.  The library's per-device set-up (the first call
 *    of any entry point on a device) looks the array up and clears it,
 *    synchronously; make one call on a device before capturing a graph.
 *  - Sharing: every launch of one class on one device uses the same region,
 *    which keeps what the last launch left (the state its class's next
 *    launch expects, so nothing needs clearing between calls).  Two such
 *    launches of one class in flight at the same time on one device (two
 *    streams, or a graph replay concurrent with a stream launch) race on
 *    the region: the caller orders them. */
#define SPMD_NOALLOC_REGION_BYTES ((1u << 20) + 16384u)
int spmd_launch_noalloc(int kernel_id, spmd_dim3 grid, spmd_dim3 block, size_t dyn_shmem, void** args,
                        void* stream);

/* Bytes of workspace a launch of `kernel_id` with this grid and block needs
 * for n elements (0 when the class needs none). */
size_t spmd_workspace_size(int kernel_id, spmd_dim3 grid, spmd_dim3 block, uint64_t n);

/* Wait for all work on `stream`, then read and clear this device's error
 * word: SPMD_ERR_DEVICE if a kernel set it since the last sync (the paper's
 * host waits on a condition variable until the queue drains, Section IV).
 * The error word is one per device, not per stream: a sync on any stream
 * reports -- and clears -- an error raised by any of the library's kernels
 * on the device since the last sync, including one raised by a kernel of
 * another stream that is still running.  A caller that needs to know which
 * stream failed synchronises one stream at a time. */
int spmd_sync(void* stream);

/* spmd_sync with a bound: polls the stream until it is idle or `ms`
 * milliseconds have passed (SPMD_ERR_TIMEOUT; the work keeps running and
 * the error word is left as it is, for a later sync to read). */
int spmd_sync_timeout(void* stream, uint32_t ms);

/* Bound on every cross-block wait of the library's kernels on the current
 * device (a scan's look-back, the reduction's final gather), in polls of
 * the awaited word; 0 restores the default (2^22 polls, seconds).  A wait
 * that reaches the bound stops waiting, treats the missing value as zero
 * and sets the device error word (SPMD_ERR_DEVICE at the next sync), so a
 * kernel whose partner blocks never publish still ends.  Set
 * synchronously; it applies to launches made after the call.  For failure
 * detection: a short bound turns a stalled wait into a prompt error. */
int spmd_set_spin_limit(uint32_t polls);

/* Parameter kinds of a class as a string, one character per args[] entry:
 * 'p' device pointer, 'u' uint32_t.  NULL for an unknown id. */
const char* spmd_kernel_signature(int kernel_id);

/* Name of a class ("reduce_i32", ...), NULL for an unknown id. */
const char* spmd_kernel_name(int kernel_id);

/* Text for a status code. */
const char* spmd_error_string(int code);

/* Text of the last HIP error seen by this thread's last failing call. */
const char* spmd_last_hip_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SPMD_H */
