// common.hpp -- internal glue shared by the runtime and the kernel-class
// translation units: the launch context handed to a class launcher, the
// kernel-side parameter unpacking (the paper's kernel prologue, Section
// III-C2: parameter i is read from the object args[i] points to), and the
// device error bits.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "spmd.h"

namespace spmd {

// Bits of the per-device error word.
enum : uint32_t {
    ERRBIT_SPIN_LIMIT = 1u,   // a cross-block wait gave up (look-back, queue)
    ERRBIT_BAD_DESC = 2u,     // a batch descriptor named an unknown class
    ERRBIT_QUEUE = 4u,        // a batch chunk fell outside its instance
};

// Fetch cursors of one batch queue segment in the run area: up to 8 chunk
// ranges, one 32-bit cursor per 128-byte slot.
constexpr size_t BATCH_CURSOR_RANGES = 8, BATCH_CURSOR_SLOT = 128;
constexpr size_t BATCH_SEG_CURSOR_BYTES = BATCH_CURSOR_RANGES * BATCH_CURSOR_SLOT;

// A device's error state, two words: [0] the error bits above, [1] the
// bound on every cross-block wait, in polls (0: DEFAULT_SPIN_LIMIT).
constexpr uint32_t DEFAULT_SPIN_LIMIT = 1u << 22;
__device__ __forceinline__ uint32_t spin_limit(const uint32_t* err) {
    const uint32_t v = err[1];
    return v ? v : DEFAULT_SPIN_LIMIT;
}

struct DevInfo {
    int device;
    int num_cus;
    size_t max_shmem_per_block;
    uint32_t* err_word;  // device address of this device's error state (two words)
    uint8_t* scratch;    // device address of this device's static scratch (noalloc.hip)
};

struct LaunchCtx {
    int kernel_id;
    spmd_dim3 grid, block;
    size_t dyn_shmem;
    void** args;
    hipStream_t stream;
    const DevInfo* dev;
};

// Kernel prologue: parameter i of the packed argument object.
template <typename T>
inline T arg(void** args, int i) {
    return *reinterpret_cast<T*>(args[i]);
}

inline bool is_pow2(uint64_t v) { return v && !(v & (v - 1)); }
inline uint32_t next_pow2(uint32_t v) {
    uint32_t p = 1;
    while (p < v) p <<= 1;
    return p;
}
inline bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }
// Do the byte ranges [a, a + na) and [b, b + nb) share a byte?
inline bool overlap(const void* a, uint64_t na, const void* b, uint64_t nb) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return na && nb && x < y + nb && y < x + na;
}

// Segment of a block in the reduce and histogram classes: S = 4*ceil(n/(4G)).
// Elements per block, a multiple of 4: 4 * ceil(n / (4 * grid)).  It fits
// 32 bits unless grid is 1 and n > 2^32 - 4; the launchers reject that.
inline uint64_t segment_len(uint32_t n, uint32_t grid) {
    return 4ull * ((n + 4ull * grid - 1) / (4ull * grid));
}

int hip_fail(hipError_t e);  // records the HIP error text, returns SPMD_ERR_HIP

// Events of a timed launch (spmd_launch_timed), null outside one.  The
// start event (if any) is bound to the launch's first kernel dispatch and
// the stop event to every dispatch, the last one standing, so the span
// between them is the device time of the launch's kernels and no marker
// packet sits between the launch and its neighbours on the stream.
struct LaunchEvents {
    hipEvent_t start, stop;
    bool used;  // a dispatch has taken them
};
extern thread_local LaunchEvents g_launch_events;

// Every kernel dispatch of spmd_launch's class launchers goes through here.
template <typename F, typename... Args>
inline void dispatch(F kernel, const dim3& grid, const dim3& block, uint32_t dyn_shmem, hipStream_t stream,
                     Args... args) {
    LaunchEvents& ev = g_launch_events;
    if (ev.stop) {
        hipExtLaunchKernelGGL(kernel, grid, block, dyn_shmem, stream, ev.used ? nullptr : ev.start, ev.stop, 0u,
                              args...);
        ev.used = true;
    } else {
        hipLaunchKernelGGL(kernel, grid, block, dyn_shmem, stream, args...);
    }
}

// The runtime keeps the error of the last failing call until it is read.
// Entry points clear one that earlier, unrelated calls (another library's)
// left behind before they launch, so the hipGetLastError after their
// launches reports those launches only.
inline void clear_stale_error() { (void)hipGetLastError(); }

// State of the current device (created on first use with the device current).
int runtime_dev(const DevInfo** out);
// Device set-up of spmd_launch_noalloc's static scratch (noalloc.hip): its
// device address on the current device, cleared.
int noalloc_setup(uint8_t** out);

// Class launchers (one translation unit each).  They validate the
// class-specific rules and enqueue the work.
int launch_reduce_i32(const LaunchCtx& c);
int launch_scan_i32(const LaunchCtx& c);
int launch_hist256_u32(const LaunchCtx& c);
int launch_jacobi5_f32(const LaunchCtx& c);
int launch_gemm_f32(const LaunchCtx& c);
int launch_warptest(const LaunchCtx& c);
int launch_reverse_i32(const LaunchCtx& c);
int launch_compact_i32(const LaunchCtx& c);
int launch_jacobi5t_f32(const LaunchCtx& c);

size_t ws_reduce_i32(spmd_dim3 grid, spmd_dim3 block, uint64_t n);

}  // namespace spmd

struct spmd_batch;
namespace spmd {
// Batch plans that are enqueued once and destroyed at once run their group
// kernels in order on the caller's stream (batch.hip).
void batch_run_in_order(spmd_batch* b);
size_t ws_scan_i32(spmd_dim3 grid, spmd_dim3 block, uint64_t n);
size_t ws_compact_i32(spmd_dim3 grid, spmd_dim3 block, uint64_t n);

}  // namespace spmd
