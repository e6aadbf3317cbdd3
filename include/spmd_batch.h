/* spmd_batch.h -- batched execution of many kernel-class instances by
 * persistent workgroups that drain a device block queue.
 *
 * This is the GPU form of the paper's runtime (Section IV): the host pushes
 * launches into a task queue, workers fetch blocks from it in chunks of
 * block_per_fetch blocks ("coarse-grained fetching", Section IV-A), and the
 * fetch itself is one atomic operation on the queue's cursor.  Here the
 * workers are resident workgroups, the cursor is a device counter advanced
 * with one relaxed device-scope atomic per fetch, and the queue is a table
 * of chunks (instance, first logical block) built on the host.  A batch is
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
 * `items` elements per thread (REDUCE, SCAN, HIST: 1, 2, 4, 8 or 16; JACOBI:
 * cells per thread down a column, 1, 2, 4 or 8, with blocks of 64 x
 * block/64 threads); `bpf` logical blocks per fetch (>= 1; a SCAN
 * instance always fetches one tile at a time, since the tiles of one fetch
 * run in sequence and its successor waits on the last of them). */
typedef struct {
    uint32_t block;
    uint32_t items;
    uint32_t bpf;
} spmd_schedule;

/* One instance.  kernel_id is SPMD_REDUCE_I32, SPMD_SCAN_I32,
 * SPMD_HIST256_U32 or SPMD_JACOBI5_F32; `n` elements (JACOBI: nx columns),
 * `ny` rows for JACOBI (1 otherwise).  `in` is x / keys / u; `out` is the
 * int32 total (REDUCE), y[n] (SCAN), the 256 uint32 bins (HIST, overwritten)
 * or u_next (JACOBI, one sweep).  `block_dim` is the blockDim the instance
 * was written for; it is a feature of the instance, not a constraint on its
 * schedule. */
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

/* Run the batch on `stream`: a prologue kernel clears the per-run state,
 * then one persistent kernel per non-empty (class, block size) queue drains
 * it. */
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

#ifdef __cplusplus
}
#endif
#endif /* SPMD_BATCH_H */
