// tune.hip -- timing of one instance under candidate schedules (spmd_tune.h).
#include <vector>

#include "common.hpp"
#include "spmd_tune.h"

using namespace spmd;

extern "C" {

size_t spmd_tune_workspace_size(const spmd_batch_item* item, const spmd_schedule* scheds, int ns) {
    if (!item || !scheds || ns <= 0) return 0;
    size_t mx = 0;
    for (int s = 0; s < ns; ++s) {
        const size_t b = spmd_batch_workspace_size(item, scheds + s, 1);
        if (b == 0) return 0;
        mx = b > mx ? b : mx;
    }
    return mx;
}

int spmd_tune_time(const spmd_batch_item* item, const spmd_schedule* scheds, int ns, uint32_t reps,
                   void* workspace, size_t ws_bytes, void* stream, float* ms_out) {
    if (!item || !scheds || ns <= 0 || reps == 0 || !ms_out) return SPMD_ERR_ARGS;
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::vector<hipEvent_t> ev(reps + 1);
    hipError_t e = hipSuccess;
    int made = 0;
    for (; made < (int)ev.size(); ++made)
        if ((e = hipEventCreate(&ev[made])) != hipSuccess) break;
    int rc = e == hipSuccess ? SPMD_OK : hip_fail(e);
    for (int s = 0; s < ns && rc == SPMD_OK; ++s) {
        spmd_batch* b = nullptr;
        if ((rc = spmd_batch_create(item, scheds + s, 1, workspace, ws_bytes, 0, &b))) break;
        rc = spmd_batch_launch(b, stream);  // warm-up
        for (uint32_t r = 0; r < reps && rc == SPMD_OK; ++r) {
            if ((e = hipEventRecord(ev[r], st)) != hipSuccess) rc = hip_fail(e);
            if (rc == SPMD_OK) rc = spmd_batch_launch(b, stream);
        }
        if (rc == SPMD_OK && (e = hipEventRecord(ev[reps], st)) != hipSuccess) rc = hip_fail(e);
        if (rc == SPMD_OK && (e = hipEventSynchronize(ev[reps])) != hipSuccess) rc = hip_fail(e);
        float best = 0.0f;
        for (uint32_t r = 0; r < reps && rc == SPMD_OK; ++r) {
            float ms = 0.0f;
            if ((e = hipEventElapsedTime(&ms, ev[r], ev[r + 1])) != hipSuccess) rc = hip_fail(e);
            if (r == 0 || ms < best) best = ms;
        }
        ms_out[s] = best;
        spmd_batch_destroy(b);
    }
    for (int i = 0; i < made; ++i) hipEventDestroy(ev[i]);
    return rc;
}

}  // extern "C"
