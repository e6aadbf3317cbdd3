/* spmd_batch.h -- batched execution of many kernel-class instances by
 * persistent workgroups that drain a device block queue.
 *
 * This is the GPU form of the paper's runtime (Section IV): the host pushes
 * launches into a task queue, workers fetch blocks from it in chunks of
 * block_per_fetch blocks ("coarse-grained fetching", Section IV-A), and the
 * fetch itself is one atomic operation on the queue's cursor.  Here the
 * workers are resident workgroups, a cursor is a device counter advanced
 * with one relaxed device-scope atomic per fetch, and the queue is a table
 * of chunks (instance, first logical block) built on the host.  A queue
 * cuts its chunks into up to 8 contiguous ranges with a cursor each
 * (workgroup w serves range w mod 8, i.e. one XCD, and moves on to the
 * other ranges once its own is drained), which spreads the fetch atomics
 * over 8 counters and keeps a range's data in one XCD's L2.  A scan queue
 * cuts only at instance starts, and only when its tiles are small (4096
 * elements or fewer on average); its tiles are all drawn, in order within
 * an instance.  A batch is
 * prepared once (spmd_batch_create: descriptors and chunk tables uploaded,
 * optional hipGraph captured) and then run any number of times.
 *
 * Instances of one batch must be independent of each other (no instance
 * reads another's output); the result of a batch is the result of running
 * each instance alone.  All conventions of spmd.h apply (status codes,
 * asynchrony, caller-owned device memory).
 */
#ifndef SPMD_BATCH_H
#define SPMD_BATCH_H

#include <stddef.h>
#include <stdint.h>

#include "spmd.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Schedule of one instance: how its work is cut into logical blocks and
 * fetched.  `block` threads per logical block (64, 128, 256 or 512);
 * `items` elements per thread (REDUCE, HIST: 1, 2, 4, 8 or 16; SCAN: also
 * 32, tiles held in registers that run in a queue of their own;
 * JACOBI: cells per thread down a column, 1, 2, 4 or 8, with blocks of
 * 64 x block/64 threads); `bpf` logical blocks per fetch (>= 1; a SCAN
 * instance always fetches one tile at a time, since the tiles of one fetch
 * run in sequence and its successor waits on the last of them).  bpf 0
 * takes the instance out of the queue: it runs as its class's own grid,
 * one logical block per workgroup, dispatched by the hardware (the choice
 * for one large instance alone in its level, e.g. a sweep of a dependent
 * stencil chain). */
typedef struct {
    uint32_t block;
    uint32_t items;
    uint32_t bpf;
} spmd_schedule;

/* One instance.  kernel_id is SPMD_REDUCE_I32, SPMD_SCAN_I32,
 * SPMD_HIST256_U32 or SPMD_JACOBI5_F32; `n` elements (JACOBI: nx columns),
 * `ny` rows for JACOBI (1 otherwise).  `in` is x / keys / u; `out` is the
 * int32 total (REDUCE), y[n] (SCAN), the 256 uint32 bins (HIST, overwritten)
 * or u_next (JACOBI, one sweep).  `out` may not overlap `in`
 * (SPMD_ERR_ARGS): a plan may run an instance more than once.  The
 * instances of one dependency level (all of them, without dependencies)
 * run concurrently and in no order, like kernels on different streams: an
 * instance's `out` must not overlap the `in` or `out` of another instance
 * of its level.  The plan does not check this; two HIST instances of one
 * level that share their bins leave the sum of both histograms there.
 * `block_dim` is the blockDim the instance was written for; it is a
 * feature of the instance, not a constraint on its schedule. */
typedef struct {
    int32_t kernel_id;
    uint32_t n;
    uint32_t ny;
    uint32_t block_dim;
    const void* in;
    void* out;
} spmd_batch_item;

typedef struct spmd_batch spmd_batch;

/* Number of logical blocks of `item` under `sched` (0 for an invalid pair). */
uint64_t spmd_batch_item_blocks(const spmd_batch_item* item, const spmd_schedule* sched);

/* Workspace bytes a batch of `n` items with these schedules needs. */
size_t spmd_batch_workspace_size(const spmd_batch_item* items, const spmd_schedule* sched, int n);

/* Validate the items, lay out `workspace` (device memory of at least
 * spmd_batch_workspace_size bytes, 256-byte aligned, owned by the caller,
 * alive until spmd_batch_destroy), upload descriptors and chunk tables
 * (synchronously) and return a plan.  `workers_per_cu` persistent
 * workgroups per compute unit and group (0 = as many as fit). */
int spmd_batch_create(const spmd_batch_item* items, const spmd_schedule* sched, int n, void* workspace,
                      size_t ws_bytes, uint32_t workers_per_cu, spmd_batch** out);

/* Dependencies between instances (the device-side counterpart of the
 * barrier inserted between an asynchronous kernel and work that reads its
 * results, Section III-C1; the queue of Section IV itself keeps no order
 * between kernels).  dep[i] is the index of an earlier instance
 * (dep[i] < i) whose results instance i reads, or SPMD_NO_DEP; a NULL `dep`
 * means none.  Instance i then sits one dependency level above dep[i]; each
 * run executes the levels one after another, every level as one persistent
 * kernel per (class, block size) queue present in it, so a chain such as
 * 100 Jacobi sweeps is one batch, one graph, and no host round trip.  An
 * instance may read from several earlier instances as long as they all sit
 * below its level (levels are ordered as a whole).  A HIST instance's bins
 * are cleared in stream order just before its own level, so an instance of
 * a lower level still reads what the bins held before.  dep[i] >= i
 * (including a self-dependency) is SPMD_ERR_ARGS.  Without dependencies the
 * result is the plain create's. */
#define SPMD_NO_DEP 0xFFFFFFFFu

size_t spmd_batch_workspace_size_dep(const spmd_batch_item* items, const spmd_schedule* sched, const uint32_t* dep,
                                     int n);

int spmd_batch_create_dep(const spmd_batch_item* items, const spmd_schedule* sched, const uint32_t* dep, int n,
                          void* workspace, size_t ws_bytes, uint32_t workers_per_cu, spmd_batch** out);

/* Run the batch on `stream`: a prologue kernel clears the per-run state,
 * then, level by level, one persistent kernel per non-empty (class, block
 * size) queue drains it. */
int spmd_batch_launch(spmd_batch* b, void* stream);

/* The same work as spmd_batch_launch, replayed from a hipGraph captured on
 * the first call. */
int spmd_batch_graph_launch(spmd_batch* b, void* stream);

/* The baseline: every instance as its own grid, one spmd_launch-equivalent
 * per instance (grid = logical block count of its schedule, hardware
 * dispatch of the blocks), issued from a host loop. */
int spmd_batch_launch_each(spmd_batch* b, void* stream);

/* Total logical blocks and chunks of the plan, and its kernel launches per
 * run of spmd_batch_launch and of spmd_batch_launch_each. */
int spmd_batch_stats(const spmd_batch* b, uint64_t* blocks, uint64_t* chunks, uint32_t* persistent_launches,
                     uint32_t* each_launches);

int spmd_batch_destroy(spmd_batch* b);

/* The worker pool of one queue on the current device: the number of
 * persistent workgroups of `block` threads a batch runs for class
 * `kernel_id` (resident workgroups per compute unit, capped at
 * workers_per_cu when non-zero, times the compute units).  Instances are
 * queued per (class, block size); each queue drains in its own persistent
 * kernel.  The paper's average coarse-grained fetching takes
 * ceil(blocks / pool) blocks per fetch (Section IV-A). */
int spmd_batch_pool_size(int kernel_id, uint32_t block, uint32_t workers_per_cu, uint32_t* pool);


/* ---- CUDA-style launch descriptors (the batch form of spmd_launch) ---- */

/* One launch as spmd_launch would take it: kernel id, grid, block, dynamic
 * shared memory bytes and the packed argument pointers (read during the
 * call only).  Batchable classes and their arguments:
 *   SPMD_REDUCE_I32   x, partials, out, n, workspace   (only `out` is written:
 *                     the batch keeps block partials in its own scratch)
 *   SPMD_SCAN_I32     x, y, n, workspace               (workspace unused)
 *   SPMD_HIST256_U32  keys, hist, n
 *   SPMD_JACOBI5_F32  u, u_next, nx, ny
 * The blockDim (product of `block`) is kept as the instance's launched
 * block size; the grid fixes the elements per thread of the as-launched
 * schedule. */
typedef struct {
    int kernel_id;
    spmd_dim3 grid, block;
    uint32_t dyn_shmem;
    void** args;
} spmd_launch_desc;

enum {
    /* blockDim as launched (rounded down to 64..512, a power of two),
     * elements per thread from grid x block, and the paper's average
     * coarse-grained fetching, ceil(blocks / pool) per fetch (Section IV-A) */
    SPMD_SCHED_AS_LAUNCHED = 0,
    /* under the loaded cost model (spmd_model_load), batch-aware: among
     * the schedules predicted within the model's slack (SPMD_BATCH_SLACK
     * unless spmd_model_batch_slack set another) of the least, the one
     * with the fewest chunks (spmd_mlp_choose_batch); launches whose
     * ensemble spread exceeds the model's threshold are tuned exhaustively
     * instead (spmd_tune_time over every candidate, fastest alone), and
     * that choice is cached by (class, sizes, blockDim) */
    SPMD_SCHED_LEARNED = 1
};

/* Default slack of the batch-aware learned choice: 20% over the least
 * predicted time buys fewer chunks to fetch (measured on the 10 000-launch
 * mixed queue: 6.3 ms against 8.8 ms for the least predicted time per
 * launch).  The best slack depends on the model; a trained model carries
 * its own, chosen on held-out launches, and sets it with
 * spmd_model_batch_slack. */
#define SPMD_BATCH_SLACK 0.2f

/* Chunk counts of n launches under every candidate schedule (the order of
 * spmd_sched_candidates): out[n x candidates], 0xFFFFFFFF where the
 * candidate is invalid for the launch.  Host only. */
int spmd_sched_chunks(const spmd_batch_item* items, int n, uint32_t* out);

/* Workspace bytes that spmd_launch_batch needs for these launches under
 * any schedule (0 if a launch is invalid for batching). */
size_t spmd_launch_batch_workspace_size(const spmd_launch_desc* descs, int n);

/* Run n independent launches as one batch on `stream` (persistent workers
 * draining the block queue).  Waits for earlier work on `stream` before
 * reusing `workspace` (device memory, 256-byte aligned, caller-owned, alive
 * until the batch completes), chooses the schedules, uploads the plan and
 * enqueues it; returns without waiting for the batch.  Results are those
 * of spmd_launch on each descriptor alone (REDUCE: `out` only).
 * SPMD_ERR_ARGS for SPMD_SCHED_LEARNED without a loaded model. */
int spmd_launch_batch(const spmd_launch_desc* descs, int n, int schedule_mode, void* workspace, size_t ws_bytes,
                      void* stream);

/* How the last spmd_launch_batch call on this thread chose its schedules. */
typedef struct {
    uint32_t launches;
    uint32_t by_model;       /* chosen by the cost model                     */
    uint32_t tuned;          /* model not confident: tuned exhaustively now  */
    uint32_t cached;         /* model not confident: earlier tuning reused   */
} spmd_batch_report;
int spmd_launch_batch_report(spmd_batch_report* out);

/* Load the cost model used by SPMD_SCHED_LEARNED on the current device:
 * k_models parameter vectors of SPMD_MLP_NPARAM floats and the input
 * normalisation (mu[12] then inv_sd[12]), host pointers copied by the
 * call; sd_threshold is the ensemble spread above which the exhaustive
 * fallback runs (INFINITY: never; a negative value: always).  Replaces an
 * earlier model and clears the tuned-schedule cache; k_models == 0 unloads
 * the model (params and norm may then be NULL).  The device copies are the
 * library's own until the next load or unload. */
int spmd_model_load(const float* params, uint32_t k_models, const float* norm, float sd_threshold);

/* Slack of SPMD_SCHED_LEARNED's batch-aware choice for the model loaded on
 * the current device: the fewest chunks among the schedules predicted
 * within ln(1 + slack) of the least (the grain-size trade-off of the
 * paper's coarse-grained fetching, Section IV-A, made per launch).
 * spmd_model_load resets it to SPMD_BATCH_SLACK.  SPMD_ERR_ARGS without a
 * loaded model, or for a negative or non-finite slack. */
int spmd_model_batch_slack(float slack);

/* The candidate schedules the tuner and the cost model range over, in
 * their fixed order (block 64..512, then items 1..32, then bpf 1..32; 144
 * in all, items 32 valid for SCAN only, items above 8 not for JACOBI);
 * writes up to `cap` of them and returns how many there are. */
uint32_t spmd_sched_candidates(spmd_schedule* out, uint32_t cap);

/* The 9 launch features of an instance as the cost model sees them: class
 * one-hot (REDUCE, SCAN, HIST, JACOBI), log2 of its elements (JACOBI:
 * nx * ny), log2 of its blockDim, log2 of the shared-memory bytes and the
 * barriers per block and warp-level operations per warp of the class's
 * block program at that blockDim. */
int spmd_sched_features(const spmd_batch_item* item, float* out9);

#ifdef __cplusplus
}
#endif
#endif /* SPMD_BATCH_H */
