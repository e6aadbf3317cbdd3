/* spmd_tune.h -- measured timings for the schedule autotuner.
 *
 * The paper picks the blocks fetched per queue access by heuristics
 * (average fetching, ceil(grid / pool), or a more aggressive count found
 * by hand; Section IV-A).  The autotuner instead measures: it runs one
 * instance alone through the persistent block queue (spmd_batch.h) under
 * each candidate schedule and records the time, which both picks the best
 * schedule exhaustively and provides the training data of the learned
 * cost model (spmd_mlp.h).
 */
#ifndef SPMD_TUNE_H
#define SPMD_TUNE_H

#include <stddef.h>
#include <stdint.h>

#include "spmd_batch.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Workspace bytes for spmd_tune_time over these schedules (the largest
 * one-instance batch among them). */
size_t spmd_tune_workspace_size(const spmd_batch_item* item, const spmd_schedule* scheds, int ns);

/* For each schedule s: build a one-instance batch in `workspace`, run it
 * once to warm up, then `reps` times, timing every run with HIP events on
 * `stream`; ms_out[s] is the fastest run in milliseconds (prologue plus
 * persistent kernel).  Synchronises `stream`.  The instance's output is
 * overwritten by every run. */
int spmd_tune_time(const spmd_batch_item* item, const spmd_schedule* scheds, int ns, uint32_t reps,
                   void* workspace, size_t ws_bytes, void* stream, float* ms_out);

#ifdef __cplusplus
}
#endif
#endif /* SPMD_TUNE_H */
