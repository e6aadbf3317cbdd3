// runtime.hip -- the C ABI declared in spmd.h: validation, dispatch to the
// class launchers, completion and error reporting.
//
// A launch mirrors the paper's push (Section IV, "Push task queue"): the
// host records grid, block, dynamic shared memory and the packed arguments
// and returns at once; the hardware dispatcher then hands workgroups to the
// compute units, which is where the paper's fetch loop runs for a single
// grid.  Synchronisation waits for the stream and then reads the device
// error word (the paper's host waits until the queue drains).
#include <stdio.h>
#include <string.h>

#include <chrono>
#include <mutex>
#include <thread>

#include "common.hpp"

namespace spmd {

// One error state per device: the error word, then the spin limit of
// cross-block waits (common.hpp).  Host code never uses this name as an
// address: the address comes from hipGetSymbolAddress with the device
// current.
__device__ uint32_t g_error_word[2];

thread_local LaunchEvents g_launch_events = {nullptr, nullptr, false};

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
DevInfo g_dev[MAX_DEVICES];
bool g_dev_ready[MAX_DEVICES];
thread_local char g_last_hip[256] = "";

struct ClassInfo {
    const char* name;
    const char* sig;
    int (*launch)(const LaunchCtx&);
    size_t (*ws)(spmd_dim3, spmd_dim3, uint64_t);
};

size_t ws_none(spmd_dim3, spmd_dim3, uint64_t) { return 0; }

const ClassInfo kClasses[SPMD_NUM_KERNELS + 1] = {
    {nullptr, nullptr, nullptr, nullptr},
    {"reduce_i32", "pppup", launch_reduce_i32, ws_reduce_i32},
    {"scan_i32", "ppup", launch_scan_i32, ws_scan_i32},
    {"hist256_u32", "ppu", launch_hist256_u32, ws_none},
    {"jacobi5_f32", "ppuu", launch_jacobi5_f32, ws_none},
    {"gemm_f32", "pppuuu", launch_gemm_f32, ws_none},
    {"warptest", "ppp", launch_warptest, ws_none},
    {"reverse_i32", "pu", launch_reverse_i32, ws_none},
    {"compact_i32", "pppuup", launch_compact_i32, ws_compact_i32},
    {"jacobi5t_f32", "ppuuu", launch_jacobi5t_f32, ws_none},
};

const ClassInfo* class_info(int id) {
    if (id < 1 || id > SPMD_NUM_KERNELS) return nullptr;
    return &kClasses[id];
}

}  // namespace

int hip_fail(hipError_t e) {
    snprintf(g_last_hip, sizeof g_last_hip, "%s: %s", hipGetErrorName(e), hipGetErrorString(e));
    return SPMD_ERR_HIP;
}

int runtime_dev(const DevInfo** out) {
    int d = 0;
    hipError_t e = hipGetDevice(&d);
    if (e != hipSuccess) return hip_fail(e);
    if (d < 0 || d >= MAX_DEVICES) return SPMD_ERR_HIP;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_dev_ready[d]) {
        DevInfo& di = g_dev[d];
        di.device = d;
        int v = 0;
        if ((e = hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, d)) != hipSuccess) return hip_fail(e);
        di.num_cus = v;
        if ((e = hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, d)) != hipSuccess) return hip_fail(e);
        di.max_shmem_per_block = (size_t)v;
        void* p = nullptr;
        if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_error_word))) != hipSuccess) return hip_fail(e);
        di.err_word = static_cast<uint32_t*>(p);
        if ((e = hipMemset(di.err_word, 0, 2 * sizeof(uint32_t))) != hipSuccess) return hip_fail(e);
        int rc = noalloc_setup(&di.scratch);
        if (rc) return rc;
        g_dev_ready[d] = true;
    }
    *out = &g_dev[d];
    return SPMD_OK;
}

static int read_and_clear_error(const DevInfo* di) {
    uint32_t v = 0;
    hipError_t e = hipMemcpy(&v, di->err_word, sizeof v, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e);
    if (v) {
        const uint32_t zero = 0;
        e = hipMemcpy(di->err_word, &zero, sizeof zero, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e);
        return SPMD_ERR_DEVICE;
    }
    return SPMD_OK;
}

}  // namespace spmd

using namespace spmd;

extern "C" {

int spmd_launch(int kernel_id, spmd_dim3 grid, spmd_dim3 block, size_t dyn_shmem, void** args, void* stream) {
    const ClassInfo* ci = class_info(kernel_id);
    if (!ci) return SPMD_ERR_INVALID_KERNEL;
    if (!grid.x || !grid.y || !grid.z || !block.x || !block.y || !block.z) return SPMD_ERR_INVALID_DIM;
    if ((uint64_t)block.x * block.y * block.z > 1024) return SPMD_ERR_INVALID_DIM;
    if ((uint64_t)grid.x * grid.y * grid.z >= (1ull << 32)) return SPMD_ERR_INVALID_DIM;
    if (!args) return SPMD_ERR_ARGS;
    const size_t nargs = strlen(ci->sig);
    for (size_t i = 0; i < nargs; ++i)
        if (!args[i]) return SPMD_ERR_ARGS;
    const DevInfo* di = nullptr;
    int rc = runtime_dev(&di);
    if (rc) return rc;
    if (dyn_shmem > di->max_shmem_per_block) return SPMD_ERR_SHMEM;
    LaunchCtx c{kernel_id, grid, block, dyn_shmem, args, static_cast<hipStream_t>(stream), di};
    clear_stale_error();
    return ci->launch(c);
}

int spmd_launch_timed(int kernel_id, spmd_dim3 grid, spmd_dim3 block, size_t dyn_shmem, void** args, void* stream,
                      void* start_event, void* stop_event) {
    if (!stop_event) return SPMD_ERR_ARGS;
    g_launch_events = {static_cast<hipEvent_t>(start_event), static_cast<hipEvent_t>(stop_event), false};
    const int rc = spmd_launch(kernel_id, grid, block, dyn_shmem, args, stream);
    const bool used = g_launch_events.used;
    g_launch_events = {nullptr, nullptr, false};
    if (rc != SPMD_OK || used) return rc;
    // nothing was enqueued: an empty span
    const hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = start_event ? hipEventRecord(static_cast<hipEvent_t>(start_event), s) : hipSuccess;
    if (e == hipSuccess) e = hipEventRecord(static_cast<hipEvent_t>(stop_event), s);
    return e == hipSuccess ? SPMD_OK : hip_fail(e);
}

size_t spmd_workspace_size(int kernel_id, spmd_dim3 grid, spmd_dim3 block, uint64_t n) {
    const ClassInfo* ci = class_info(kernel_id);
    return ci ? ci->ws(grid, block, n) : 0;
}

int spmd_sync(void* stream) {
    const DevInfo* di = nullptr;
    int rc = runtime_dev(&di);
    if (rc) return rc;
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e);
    return read_and_clear_error(di);
}

int spmd_sync_timeout(void* stream, uint32_t ms) {
    const DevInfo* di = nullptr;
    int rc = runtime_dev(&di);
    if (rc) return rc;
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        hipError_t e = hipStreamQuery(static_cast<hipStream_t>(stream));
        if (e == hipSuccess) break;
        if (e != hipErrorNotReady) return hip_fail(e);
        const auto dt = std::chrono::steady_clock::now() - t0;
        if (std::chrono::duration_cast<std::chrono::milliseconds>(dt).count() >= (long long)ms) return SPMD_ERR_TIMEOUT;
        std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
    return read_and_clear_error(di);
}

int spmd_set_spin_limit(uint32_t polls) {
    const DevInfo* di = nullptr;
    int rc = runtime_dev(&di);
    if (rc) return rc;
    hipError_t e = hipMemcpy(di->err_word + 1, &polls, sizeof polls, hipMemcpyHostToDevice);
    return e == hipSuccess ? SPMD_OK : hip_fail(e);
}

const char* spmd_kernel_signature(int kernel_id) {
    const ClassInfo* ci = class_info(kernel_id);
    return ci ? ci->sig : nullptr;
}

const char* spmd_kernel_name(int kernel_id) {
    const ClassInfo* ci = class_info(kernel_id);
    return ci ? ci->name : nullptr;
}

const char* spmd_error_string(int code) {
    switch (code) {
    case SPMD_OK: return "ok";
    case SPMD_ERR_INVALID_KERNEL: return "invalid kernel id";
    case SPMD_ERR_INVALID_DIM: return "invalid launch dimensions for this kernel class";
    case SPMD_ERR_SHMEM: return "invalid dynamic shared memory size";
    case SPMD_ERR_ARGS: return "invalid arguments";
    case SPMD_ERR_HIP: return "HIP runtime error";
    case SPMD_ERR_DEVICE: return "a kernel reported a device-side error";
    case SPMD_ERR_TIMEOUT: return "timed out waiting for the stream";
    case SPMD_ERR_WORKSPACE: return "workspace missing, too small or misaligned";
    default: return "unknown status";
    }
}

const char* spmd_last_hip_error(void) { return g_last_hip; }

}  // extern "C"
