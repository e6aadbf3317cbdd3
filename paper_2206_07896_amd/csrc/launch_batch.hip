// launch_batch.hip -- spmd_launch_batch: CUDA-style launch descriptors run
// as one batch of the block queue, with the schedule of every launch taken
// either as launched (the paper's average coarse-grained fetching) or from
// the learned cost model, which falls back to exhaustive tuning where its
// ensemble disagrees.  Also the schedule candidates and launch features
// the tuner and the model share.
#include <math.h>
#include <string.h>

#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "common.hpp"
#include "spmd_batch.h"
#include "spmd_mlp.h"
#include "spmd_tune.h"

using namespace spmd;

namespace spmd {
// A batch instance whose output overlaps its input (batch.hip; refused with
// SPMD_ERR_ARGS).
bool batch_out_overlaps_in(const spmd_batch_item& it);
}  // namespace spmd

namespace {

constexpr uint32_t CAND_BLOCKS[4] = {64, 128, 256, 512};
constexpr uint32_t CAND_ITEMS[6] = {1, 2, 4, 8, 16, 32};
constexpr uint32_t CAND_BPF[6] = {1, 2, 4, 8, 16, 32};
constexpr uint32_t NCANDS = 4 * 6 * 6;
static_assert(NCANDS <= SPMD_MLP_MAX_CANDS, "candidate table fits the choice kernel");

spmd_schedule candidate(uint32_t j) {
    return {CAND_BLOCKS[j / 36], CAND_ITEMS[(j / 6) % 6], CAND_BPF[j % 6]};
}

// Jacobi takes at most 8 cells per thread; 32 items are scan tiles only
// (register-resident, in a queue class of their own).
bool candidate_valid(int kernel_id, const spmd_schedule& s) {
    if (s.items > 16 && kernel_id != SPMD_SCAN_I32) return false;
    return !(kernel_id == SPMD_JACOBI5_F32 && s.items > 8);
}

uint64_t cdiv64(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
size_t align256(size_t v) { return (v + 255) / 256 * 256; }

using CacheKey = std::tuple<int, uint32_t, uint32_t, uint32_t>;  // class, n, ny, blockDim

struct Model {
    float* params = nullptr;  // device, k * NPARAM
    float* norm = nullptr;    // device, 2 * DIN
    uint32_t k = 0;
    float tau = INFINITY;
    float slack = SPMD_BATCH_SLACK;  // of the batch-aware choice
    std::map<CacheKey, spmd_schedule> tuned;
};

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
Model g_model[MAX_DEVICES];
thread_local spmd_batch_report g_report = {0, 0, 0, 0};

// Launch descriptor -> batch item.
int to_item(const spmd_launch_desc& d, spmd_batch_item* it) {
    if (!d.args) return SPMD_ERR_ARGS;
    const uint64_t bd = (uint64_t)d.block.x * d.block.y * d.block.z;
    if (!d.grid.x || !d.grid.y || !d.grid.z || bd == 0 || bd > 1024) return SPMD_ERR_INVALID_DIM;
    memset(it, 0, sizeof *it);
    it->kernel_id = d.kernel_id;
    it->block_dim = (uint32_t)bd;
    it->ny = 1;
    void** a = d.args;
    switch (d.kernel_id) {
    case SPMD_REDUCE_I32:
        if (!a[0] || !a[2] || !a[3]) return SPMD_ERR_ARGS;
        it->in = arg<const void*>(a, 0);
        it->out = arg<void*>(a, 2);
        it->n = arg<uint32_t>(a, 3);
        break;
    case SPMD_SCAN_I32:
        if (!a[0] || !a[1] || !a[2]) return SPMD_ERR_ARGS;
        it->in = arg<const void*>(a, 0);
        it->out = arg<void*>(a, 1);
        it->n = arg<uint32_t>(a, 2);
        break;
    case SPMD_HIST256_U32:
        if (!a[0] || !a[1] || !a[2]) return SPMD_ERR_ARGS;
        it->in = arg<const void*>(a, 0);
        it->out = arg<void*>(a, 1);
        it->n = arg<uint32_t>(a, 2);
        break;
    case SPMD_JACOBI5_F32:
        if (!a[0] || !a[1] || !a[2] || !a[3]) return SPMD_ERR_ARGS;
        it->in = arg<const void*>(a, 0);
        it->out = arg<void*>(a, 1);
        it->n = arg<uint32_t>(a, 2);
        it->ny = arg<uint32_t>(a, 3);
        break;
    default: return SPMD_ERR_INVALID_KERNEL;
    }
    return SPMD_OK;
}

// The paper's schedule for a launch as written: its blockDim (rounded down
// to a queue block size), the elements per thread its grid implies, and
// average coarse-grained fetching over the queue's worker pool.
int as_launched(const spmd_launch_desc& d, const spmd_batch_item& it, spmd_schedule* s) {
    uint32_t bs = 64;
    while (bs < 512 && 2 * bs <= it.block_dim) bs *= 2;
    const uint64_t threads = (uint64_t)d.grid.x * d.grid.y * d.grid.z * it.block_dim;
    const uint64_t elems = it.kernel_id == SPMD_JACOBI5_F32 ? (uint64_t)it.n * it.ny : (uint64_t)it.n;
    const uint64_t per = elems ? cdiv64(elems, threads) : 1;
    const uint32_t cap = it.kernel_id == SPMD_JACOBI5_F32 ? 8u : 16u;
    uint32_t items = 1;
    while (items < cap && items < per) items *= 2;
    spmd_schedule one{bs, items, 1};
    const uint64_t nb = spmd_batch_item_blocks(&it, &one);
    if (nb == 0) return SPMD_ERR_INVALID_DIM;
    uint32_t pool = 0;
    int rc = spmd_batch_pool_size(it.kernel_id, bs, 0, &pool);
    if (rc) return rc;
    const uint64_t bpf = cdiv64(nb, pool ? pool : 1);
    *s = {bs, items, (uint32_t)(bpf < 1 ? 1 : (bpf > 0xFFFFFFFFull ? 0xFFFFFFFFu : bpf))};
    return SPMD_OK;
}

// Bound on the batch workspace over every schedule: the finest schedule
// (64 threads, 1 item, 1 block per fetch) has the most blocks and chunks;
// each further queue group (20 at most: 5 queue classes -- the wide scan
// included -- x 4 block sizes) can add its cursors and one 256-byte
// alignment gap.
size_t batch_bound(const std::vector<spmd_batch_item>& items) {
    std::vector<spmd_schedule> fine(items.size(), spmd_schedule{64, 1, 1});
    const size_t b = spmd_batch_workspace_size(items.data(), fine.data(), (int)items.size());
    return b ? b + 20 * (BATCH_SEG_CURSOR_BYTES + 256) : 0;
}

struct InferLayout {
    size_t cands, feats, valid, chunks, best, pred, sd, total;
};
InferLayout infer_layout(size_t n) {
    InferLayout L;
    L.cands = 0;
    L.feats = align256(L.cands + 4 * SPMD_MLP_NSCHED * NCANDS);
    L.valid = align256(L.feats + 4 * SPMD_MLP_NFEAT * n);
    L.chunks = align256(L.valid + NCANDS * n);
    L.best = align256(L.chunks + 4 * NCANDS * n);
    L.pred = align256(L.best + 4 * n);
    L.sd = align256(L.pred + 4 * n);
    L.total = align256(L.sd + 4 * n);
    return L;
}

int current_device(int* d) {
    hipError_t e = hipGetDevice(d);
    if (e != hipSuccess) return hip_fail(e);
    return (*d >= 0 && *d < MAX_DEVICES) ? SPMD_OK : SPMD_ERR_HIP;
}

// Chunks of one launch under candidate j in the block queue: its logical
// blocks, fetched bpf at a time (SCAN one tile at a time); 0xFFFFFFFF where
// the candidate is invalid for the launch.
uint32_t candidate_chunks(const spmd_batch_item& it, uint32_t j) {
    const spmd_schedule c = candidate(j);
    if (!candidate_valid(it.kernel_id, c)) return 0xFFFFFFFFu;
    const uint64_t nb = spmd_batch_item_blocks(&it, &c);
    if (nb == 0) return 0xFFFFFFFFu;
    const uint64_t bpf = it.kernel_id == SPMD_SCAN_I32 ? 1u : c.bpf;
    const uint64_t ch = (nb + bpf - 1) / bpf;
    return ch < 0xFFFFFFFFull ? (uint32_t)ch : 0xFFFFFFFEu;
}

}  // namespace

extern "C" {

int spmd_sched_chunks(const spmd_batch_item* items, int n, uint32_t* out) {
    if (n < 0 || (n && (!items || !out))) return SPMD_ERR_ARGS;
    for (int i = 0; i < n; ++i)
        for (uint32_t j = 0; j < NCANDS; ++j) out[(size_t)NCANDS * i + j] = candidate_chunks(items[i], j);
    return SPMD_OK;
}

uint32_t spmd_sched_candidates(spmd_schedule* out, uint32_t cap) {
    for (uint32_t j = 0; out && j < cap && j < NCANDS; ++j) out[j] = candidate(j);
    return NCANDS;
}

int spmd_sched_features(const spmd_batch_item* it, float* f) {
    if (!it || !f) return SPMD_ERR_ARGS;
    const int k = it->kernel_id;
    const double bd = it->block_dim ? (double)it->block_dim : 1.0;
    double elems = k == SPMD_JACOBI5_F32 ? (double)it->n * (double)it->ny : (double)it->n;
    if (elems < 1.0) elems = 1.0;
    double shm, bar, wops = 0.0;
    switch (k) {
    case SPMD_REDUCE_I32: shm = 4.0 * bd; bar = log2(bd) + 1.0; break;            // tree levels + load
    case SPMD_SCAN_I32: shm = 4.0 * floor(bd / 32.0) + 4.0; bar = 2.0; wops = 10.0; break;  // 2 x 5 shfl_up
    case SPMD_HIST256_U32: shm = 1024.0; bar = 2.0; break;                         // clear, count
    case SPMD_JACOBI5_F32: shm = 4.0 * (floor(bd / 64.0) + 2.0) * 66.0; bar = 1.0; break;  // halo tile
    default: return SPMD_ERR_INVALID_KERNEL;
    }
    f[0] = k == SPMD_REDUCE_I32 ? 1.0f : 0.0f;
    f[1] = k == SPMD_SCAN_I32 ? 1.0f : 0.0f;
    f[2] = k == SPMD_HIST256_U32 ? 1.0f : 0.0f;
    f[3] = k == SPMD_JACOBI5_F32 ? 1.0f : 0.0f;
    f[4] = (float)log2(elems);
    f[5] = (float)log2(bd);
    f[6] = (float)log2(shm);
    f[7] = (float)bar;
    f[8] = (float)wops;
    return SPMD_OK;
}

int spmd_model_load(const float* params, uint32_t k_models, const float* norm, float sd_threshold) {
    if (k_models > SPMD_MLP_MAX_MODELS || (k_models && (!params || !norm || isnan(sd_threshold))))
        return SPMD_ERR_ARGS;
    int d = 0;
    int rc = current_device(&d);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    Model& m = g_model[d];
    hipError_t e = hipSuccess;
    if (m.params) e = hipFree(m.params);
    if (e == hipSuccess && m.norm) e = hipFree(m.norm);
    m.params = nullptr;
    m.norm = nullptr;
    m.k = 0;
    m.slack = SPMD_BATCH_SLACK;
    m.tuned.clear();
    if (e != hipSuccess) return hip_fail(e);
    if (!k_models) return SPMD_OK;  // unloaded
    const size_t pb = (size_t)k_models * SPMD_MLP_NPARAM * sizeof(float), nb = 2 * SPMD_MLP_DIN * sizeof(float);
    if ((e = hipMalloc(&m.params, pb)) != hipSuccess) return hip_fail(e);
    if ((e = hipMalloc(&m.norm, nb)) != hipSuccess) return hip_fail(e);
    if ((e = hipMemcpy(m.params, params, pb, hipMemcpyHostToDevice)) != hipSuccess) return hip_fail(e);
    if ((e = hipMemcpy(m.norm, norm, nb, hipMemcpyHostToDevice)) != hipSuccess) return hip_fail(e);
    m.k = k_models;
    m.tau = sd_threshold;
    return SPMD_OK;
}

int spmd_model_batch_slack(float slack) {
    if (!(slack >= 0.0f) || !(slack < 1e30f)) return SPMD_ERR_ARGS;
    int d = 0;
    int rc = current_device(&d);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    Model& m = g_model[d];
    if (!m.k) return SPMD_ERR_ARGS;
    m.slack = slack;
    return SPMD_OK;
}

size_t spmd_launch_batch_workspace_size(const spmd_launch_desc* descs, int n) {
    if (!descs || n <= 0) return 0;
    std::vector<spmd_batch_item> items(n);
    for (int i = 0; i < n; ++i)
        if (to_item(descs[i], &items[i]) != SPMD_OK) return 0;
    const size_t b = batch_bound(items);
    if (!b) return 0;
    const size_t inf = infer_layout((size_t)n).total;
    return b > inf ? b : inf;
}

int spmd_launch_batch_report(spmd_batch_report* out) {
    if (!out) return SPMD_ERR_ARGS;
    *out = g_report;
    return SPMD_OK;
}

int spmd_launch_batch(const spmd_launch_desc* descs, int n, int mode, void* workspace, size_t ws_bytes,
                      void* stream) {
    g_report = {0, 0, 0, 0};
    if (!descs || n <= 0 || (mode != SPMD_SCHED_AS_LAUNCHED && mode != SPMD_SCHED_LEARNED)) return SPMD_ERR_ARGS;
    std::vector<spmd_batch_item> items(n);
    int rc;
    for (int i = 0; i < n; ++i) {
        if ((rc = to_item(descs[i], &items[i]))) return rc;
        if (batch_out_overlaps_in(items[i])) return SPMD_ERR_ARGS;
    }
    const size_t bound = batch_bound(items);
    if (!bound) return SPMD_ERR_INVALID_DIM;
    const InferLayout IL = infer_layout((size_t)n);
    if (!workspace || ((uintptr_t)workspace % 256) || ws_bytes < bound || ws_bytes < IL.total)
        return SPMD_ERR_WORKSPACE;
    int dev = 0;
    if ((rc = current_device(&dev))) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = hipStreamSynchronize(st);  // the workspace may still be read by the previous batch
    if (e != hipSuccess) return hip_fail(e);

    std::vector<spmd_schedule> sched(n);
    spmd_batch_report rep = {(uint32_t)n, 0, 0, 0};
    if (mode == SPMD_SCHED_AS_LAUNCHED) {
        for (int i = 0; i < n; ++i)
            if ((rc = as_launched(descs[i], items[i], &sched[i]))) return rc;
    } else {
        std::lock_guard<std::mutex> lk(g_mu);
        Model& m = g_model[dev];
        if (!m.k) return SPMD_ERR_ARGS;
        std::vector<float> cands(SPMD_MLP_NSCHED * NCANDS), feats((size_t)SPMD_MLP_NFEAT * n);
        std::vector<uint8_t> valid((size_t)NCANDS * n);
        std::vector<uint32_t> chunks((size_t)NCANDS * n);
        for (uint32_t j = 0; j < NCANDS; ++j) {
            const spmd_schedule c = candidate(j);
            cands[3 * j + 0] = (float)log2((double)c.block);
            cands[3 * j + 1] = (float)log2((double)c.items);
            cands[3 * j + 2] = (float)log2((double)c.bpf);
        }
        for (int i = 0; i < n; ++i) {
            if ((rc = spmd_sched_features(&items[i], &feats[(size_t)SPMD_MLP_NFEAT * i]))) return rc;
            for (uint32_t j = 0; j < NCANDS; ++j) {
                valid[(size_t)NCANDS * i + j] = candidate_valid(items[i].kernel_id, candidate(j)) ? 1 : 0;
                chunks[(size_t)NCANDS * i + j] = candidate_chunks(items[i], j);
            }
        }
        uint8_t* ws = static_cast<uint8_t*>(workspace);
        e = hipMemcpyAsync(ws + IL.cands, cands.data(), 4 * cands.size(), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(ws + IL.feats, feats.data(), 4 * feats.size(), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(ws + IL.valid, valid.data(), valid.size(), hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ws + IL.chunks, chunks.data(), 4 * chunks.size(), hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return hip_fail(e);
        rc = spmd_mlp_choose_batch(m.params, m.k, m.norm, reinterpret_cast<const float*>(ws + IL.feats), (uint32_t)n,
                                   reinterpret_cast<const float*>(ws + IL.cands), NCANDS, ws + IL.valid,
                                   reinterpret_cast<const uint32_t*>(ws + IL.chunks), m.slack,
                                   reinterpret_cast<uint32_t*>(ws + IL.best), reinterpret_cast<float*>(ws + IL.pred),
                                   reinterpret_cast<float*>(ws + IL.sd), stream);
        if (rc) return rc;
        std::vector<uint32_t> best(n);
        std::vector<float> sd(n);
        e = hipMemcpyAsync(best.data(), ws + IL.best, 4 * (size_t)n, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(sd.data(), ws + IL.sd, 4 * (size_t)n, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e);
        for (int i = 0; i < n; ++i) {
            if (best[i] >= NCANDS) return SPMD_ERR_INVALID_DIM;
            if (!(sd[i] > m.tau)) {
                sched[i] = candidate(best[i]);
                ++rep.by_model;
                continue;
            }
            const CacheKey key{items[i].kernel_id, items[i].n, items[i].ny, items[i].block_dim};
            auto hit = m.tuned.find(key);
            if (hit != m.tuned.end()) {
                sched[i] = hit->second;
                ++rep.cached;
                continue;
            }
            std::vector<spmd_schedule> list;
            for (uint32_t j = 0; j < NCANDS; ++j)
                if (candidate_valid(items[i].kernel_id, candidate(j))) list.push_back(candidate(j));
            if (spmd_tune_workspace_size(&items[i], list.data(), (int)list.size()) > ws_bytes)
                return SPMD_ERR_WORKSPACE;
            std::vector<float> ms(list.size());
            if ((rc = spmd_tune_time(&items[i], list.data(), (int)list.size(), 2, workspace, ws_bytes, stream,
                                     ms.data())))
                return rc;
            size_t arg = 0;
            for (size_t j = 1; j < list.size(); ++j)
                if (ms[j] < ms[arg]) arg = j;  // ties go to the earlier candidate
            sched[i] = list[arg];
            m.tuned[key] = list[arg];
            ++rep.tuned;
        }
    }
    spmd_batch* b = nullptr;
    if ((rc = spmd_batch_create(items.data(), sched.data(), n, workspace, ws_bytes, 0, &b))) return rc;
    batch_run_in_order(b);
    rc = spmd_batch_launch(b, stream);
    spmd_batch_destroy(b);  // host plan only: the device tables stay in the workspace
    if (rc == SPMD_OK) g_report = rep;
    return rc;
}

}  // extern "C"
