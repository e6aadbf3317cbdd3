// mlp.hip -- kernels of the schedule cost model (spmd_mlp.h).
//
// Forward: one thread per row, the parameters staged in LDS (every lane
// reads the same weight at the same time: LDS broadcast).  Backward: a
// block of 64 rows keeps their inputs, activations and back-propagated
// errors in LDS and forms its partial weight gradients with sums over its
// rows in row order; a second kernel adds the block partials in block
// order.  Nothing depends on scheduling, so gradients are reproducible.
#include "common.hpp"
#include "spmd_mlp.h"

namespace spmd {

constexpr int DIN = SPMD_MLP_DIN, HID = SPMD_MLP_H, NP = SPMD_MLP_NPARAM;
constexpr int OFF_W1 = 0, OFF_B1 = DIN * HID, OFF_W2 = OFF_B1 + HID, OFF_B2 = OFF_W2 + HID * HID,
              OFF_W3 = OFF_B2 + HID, OFF_B3 = OFF_W3 + HID;
static_assert(OFF_B3 + 1 == NP, "parameter layout");
constexpr int MLP_ROWS = 64;  // rows per block in forward and backward

__device__ __forceinline__ void stage_params(float* P, const float* params) {
    for (int i = threadIdx.x; i < NP; i += blockDim.x) P[i] = params[i];
}

// One row: normalised inputs -> h1 (registers) -> h2 -> y.
template <bool STORE>
__device__ __forceinline__ float row_forward(const float* P, const float* nm, const float* xrow, uint32_t i,
                                             uint32_t n, float* h1t, float* h2t) {
#pragma clang fp contract(fast)
    float xn[DIN];
#pragma unroll
    for (int k = 0; k < DIN; ++k) xn[k] = (xrow[k] - nm[k]) * nm[DIN + k];
    float h1[HID];
#pragma unroll
    for (int j = 0; j < HID; ++j) {
        float z = P[OFF_B1 + j];
#pragma unroll
        for (int k = 0; k < DIN; ++k) z += xn[k] * P[OFF_W1 + k * HID + j];
        h1[j] = z > 0.0f ? z : 0.0f;
        if (STORE) h1t[(uint64_t)j * n + i] = h1[j];
    }
    float y = P[OFF_B3];
    for (int j = 0; j < HID; ++j) {
        float z = P[OFF_B2 + j];
#pragma unroll
        for (int a = 0; a < HID; ++a) z += h1[a] * P[OFF_W2 + a * HID + j];
        const float h2 = z > 0.0f ? z : 0.0f;
        if (STORE) h2t[(uint64_t)j * n + i] = h2;
        y += h2 * P[OFF_W3 + j];
    }
    return y;
}

__global__ __launch_bounds__(MLP_ROWS) void mlp_forward_kernel(const float* __restrict__ params,
                                                               const float* __restrict__ norm,
                                                               const float* __restrict__ x, uint32_t n,
                                                               float* __restrict__ y, float* h1t, float* h2t) {
    __shared__ float P[NP];
    __shared__ float nm[2 * DIN];
    stage_params(P, params);
    if (threadIdx.x < 2 * DIN) nm[threadIdx.x] = norm[threadIdx.x];
    __syncthreads();
    const uint32_t i = blockIdx.x * MLP_ROWS + threadIdx.x;
    if (i >= n) return;
    const float* xrow = x + (uint64_t)i * DIN;
    y[i] = h1t ? row_forward<true>(P, nm, xrow, i, n, h1t, h2t) : row_forward<false>(P, nm, xrow, i, n, h1t, h2t);
}

// Block partials: part[b * (NP + 1) + p] for parameter p, the block's sum
// of squared errors at p = NP.
__global__ __launch_bounds__(MLP_ROWS) void mlp_backward_kernel(
    const float* __restrict__ params, const float* __restrict__ norm, const float* __restrict__ x,
    const float* __restrict__ t, uint32_t n, const float* __restrict__ y, const float* __restrict__ h1t,
    const float* __restrict__ h2t, float* __restrict__ part) {
#pragma clang fp contract(fast)
    __shared__ float W2[HID * HID];
    __shared__ float w3[HID];
    __shared__ float xs[MLP_ROWS][DIN];
    __shared__ float h1s[MLP_ROWS][HID + 1];
    __shared__ float h2s[MLP_ROWS][HID + 1];
    __shared__ float d2s[MLP_ROWS][HID + 1];
    __shared__ float d1s[MLP_ROWS][HID + 1];
    __shared__ float dys[MLP_ROWS];
    __shared__ float e2s[MLP_ROWS];
    const uint32_t r = threadIdx.x;
    for (int q = r; q < HID * HID; q += MLP_ROWS) W2[q] = params[OFF_W2 + q];
    w3[r] = params[OFF_W3 + r];
    __syncthreads();
    const uint32_t i = blockIdx.x * MLP_ROWS + r;
    const bool ok = i < n;
    const float err = ok ? y[i] - t[i] : 0.0f;
    const float dy = 2.0f * err / (float)n;
    dys[r] = dy;
    e2s[r] = err * err;
#pragma unroll
    for (int k = 0; k < DIN; ++k) xs[r][k] = ok ? (x[(uint64_t)i * DIN + k] - norm[k]) * norm[DIN + k] : 0.0f;
    float d2[HID];
#pragma unroll
    for (int j = 0; j < HID; ++j) {
        const float h1 = ok ? h1t[(uint64_t)j * n + i] : 0.0f;
        const float h2 = ok ? h2t[(uint64_t)j * n + i] : 0.0f;
        h1s[r][j] = h1;
        h2s[r][j] = h2;
        d2[j] = h2 > 0.0f ? dy * w3[j] : 0.0f;
        d2s[r][j] = d2[j];
    }
    for (int a = 0; a < HID; ++a) {
        float s = 0.0f;
#pragma unroll
        for (int j = 0; j < HID; ++j) s += d2[j] * W2[a * HID + j];
        d1s[r][a] = h1s[r][a] > 0.0f ? s : 0.0f;
    }
    __syncthreads();
    float* out = part + (uint64_t)blockIdx.x * (NP + 1);
    for (int p = r; p <= NP; p += MLP_ROWS) {
        float s = 0.0f;
        if (p < OFF_B1) {  // W1[k][a]
            const int k = p / HID, a = p % HID;
            for (int q = 0; q < MLP_ROWS; ++q) s += xs[q][k] * d1s[q][a];
        } else if (p < OFF_W2) {
            const int a = p - OFF_B1;
            for (int q = 0; q < MLP_ROWS; ++q) s += d1s[q][a];
        } else if (p < OFF_B2) {  // W2[a][j]
            const int a = (p - OFF_W2) / HID, j = (p - OFF_W2) % HID;
            for (int q = 0; q < MLP_ROWS; ++q) s += h1s[q][a] * d2s[q][j];
        } else if (p < OFF_W3) {
            const int j = p - OFF_B2;
            for (int q = 0; q < MLP_ROWS; ++q) s += d2s[q][j];
        } else if (p < OFF_B3) {
            const int j = p - OFF_W3;
            for (int q = 0; q < MLP_ROWS; ++q) s += dys[q] * h2s[q][j];
        } else if (p == OFF_B3) {
            for (int q = 0; q < MLP_ROWS; ++q) s += dys[q];
        } else {
            for (int q = 0; q < MLP_ROWS; ++q) s += e2s[q];
        }
        out[p] = s;
    }
}

__global__ __launch_bounds__(256) void mlp_reduce_kernel(const float* __restrict__ part, uint32_t nblocks,
                                                         uint32_t n, float* __restrict__ grad,
                                                         float* __restrict__ loss) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p > NP) return;
    float s = 0.0f;
    for (uint32_t b = 0; b < nblocks; ++b) s += part[(uint64_t)b * (NP + 1) + p];
    if (p < NP) grad[p] = s;
    else *loss = s / (float)n;
}

__global__ __launch_bounds__(256) void mlp_adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                                                       float* __restrict__ m, float* __restrict__ v, float lr,
                                                       float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= NP) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// One launch per loop iteration of a block; thread j evaluates candidate j
// under every model.
__global__ __launch_bounds__(SPMD_MLP_MAX_CANDS) void mlp_choose_kernel(
    const float* __restrict__ params, uint32_t k_models, const float* __restrict__ norm,
    const float* __restrict__ feats, uint32_t m, const float* __restrict__ cands, uint32_t c,
    const uint8_t* __restrict__ valid, const uint32_t* __restrict__ chunks, float log_slack,
    uint32_t* __restrict__ best, float* __restrict__ best_pred, float* __restrict__ best_sd) {
    extern __shared__ float P[];  // k_models * NP
    __shared__ float nm[2 * DIN];
    __shared__ float red_v[SPMD_MLP_MAX_CANDS];
    __shared__ uint32_t red_i[SPMD_MLP_MAX_CANDS];
    __shared__ float red_s[SPMD_MLP_MAX_CANDS];
    __shared__ uint32_t red_c[SPMD_MLP_MAX_CANDS];
    for (uint32_t q = threadIdx.x; q < k_models * NP; q += blockDim.x) P[q] = params[q];
    if (threadIdx.x < 2 * DIN) nm[threadIdx.x] = norm[threadIdx.x];
    __syncthreads();
    const uint32_t j = threadIdx.x;
    for (uint32_t li = blockIdx.x; li < m; li += gridDim.x) {
        float mean = INFINITY, sd = 0.0f;
        const bool ok = j < c && valid[(uint64_t)li * c + j] != 0;
        if (ok) {
            float xrow[DIN];
#pragma unroll
            for (int q = 0; q < SPMD_MLP_NFEAT; ++q) xrow[q] = feats[(uint64_t)li * SPMD_MLP_NFEAT + q];
#pragma unroll
            for (int q = 0; q < SPMD_MLP_NSCHED; ++q) xrow[SPMD_MLP_NFEAT + q] = cands[j * SPMD_MLP_NSCHED + q];
            // two passes (mean, then squared deviations): the spread of
            // nearly equal predictions keeps its precision
            float pr[SPMD_MLP_MAX_MODELS];
            float s1 = 0.0f;
#pragma unroll
            for (uint32_t mk = 0; mk < SPMD_MLP_MAX_MODELS; ++mk) {
                pr[mk] = mk < k_models ? row_forward<false>(P + mk * NP, nm, xrow, 0, 0, nullptr, nullptr) : 0.0f;
                s1 += pr[mk];
            }
            mean = s1 / (float)k_models;
            float s2 = 0.0f;
#pragma unroll
            for (uint32_t mk = 0; mk < SPMD_MLP_MAX_MODELS; ++mk) {
                const float d = pr[mk] - mean;
                s2 += mk < k_models ? d * d : 0.0f;
            }
            sd = sqrtf(s2 / (float)k_models);
        }
        red_v[j] = mean;
        red_i[j] = ok ? j : 0xFFFFFFFFu;
        red_s[j] = sd;
        __syncthreads();
        for (uint32_t w = blockDim.x / 2; w > 0; w >>= 1) {
            if (j < w) {
                const float a = red_v[j], b = red_v[j + w];
                const uint32_t ia = red_i[j], ib = red_i[j + w];
                // smaller mean wins; equal means go to the lower index
                if (b < a || (b == a && ib < ia)) {
                    red_v[j] = b;
                    red_i[j] = ib;
                    red_s[j] = red_s[j + w];
                }
            }
            __syncthreads();
        }
        if (chunks) {
            // Batch-aware second pass: among the candidates whose mean is
            // within log_slack of the least, the fewest chunks wins (then
            // the smaller mean, then the lower index).
            const float thr = red_v[0] + log_slack;
            __syncthreads();  // every thread has read red_v[0]
            const bool near = ok && mean <= thr;
            red_c[j] = near ? chunks[(uint64_t)li * c + j] : 0xFFFFFFFFu;
            red_v[j] = near ? mean : INFINITY;
            red_i[j] = near ? j : 0xFFFFFFFFu;
            red_s[j] = sd;
            __syncthreads();
            for (uint32_t w = blockDim.x / 2; w > 0; w >>= 1) {
                if (j < w) {
                    const uint32_t ca = red_c[j], cb = red_c[j + w];
                    const float a = red_v[j], b = red_v[j + w];
                    const uint32_t ia = red_i[j], ib = red_i[j + w];
                    if (cb < ca || (cb == ca && (b < a || (b == a && ib < ia)))) {
                        red_c[j] = cb;
                        red_v[j] = b;
                        red_i[j] = ib;
                        red_s[j] = red_s[j + w];
                    }
                }
                __syncthreads();
            }
        }
        if (j == 0) {
            best[li] = red_i[0];
            best_pred[li] = red_v[0];
            best_sd[li] = red_s[0];
        }
        __syncthreads();
    }
}

}  // namespace spmd

using namespace spmd;

namespace {
int choose_impl(const float* params, uint32_t k_models, const float* norm, const float* feats, uint32_t m,
                const float* cands, uint32_t c, const uint8_t* valid, const uint32_t* chunks, float log_slack,
                uint32_t* best, float* best_pred, float* best_sd, void* stream);
}  // namespace

extern "C" {

int spmd_mlp_forward(const float* params, const float* norm, const float* x, uint32_t n, float* y, float* h1t,
                     float* h2t, void* stream) {
    if (!params || !norm || (n && (!x || !y)) || (!h1t) != (!h2t)) return SPMD_ERR_ARGS;
    if (!n) return SPMD_OK;
    clear_stale_error();
    hipLaunchKernelGGL(mlp_forward_kernel, dim3((n + MLP_ROWS - 1) / MLP_ROWS), dim3(MLP_ROWS), 0,
                       static_cast<hipStream_t>(stream), params, norm, x, n, y, h1t, h2t);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SPMD_OK : hip_fail(e);
}

size_t spmd_mlp_workspace_size(uint32_t n) {
    const size_t nb = (n + MLP_ROWS - 1) / MLP_ROWS;
    return (nb ? nb : 1) * (NP + 1) * sizeof(float);
}

int spmd_mlp_backward(const float* params, const float* norm, const float* x, const float* t, uint32_t n,
                      const float* y, const float* h1t, const float* h2t, float* grad, float* loss, void* workspace,
                      size_t ws_bytes, void* stream) {
    if (!params || !norm || !x || !t || !y || !h1t || !h2t || !grad || !loss || n == 0) return SPMD_ERR_ARGS;
    if (!workspace || ws_bytes < spmd_mlp_workspace_size(n)) return SPMD_ERR_WORKSPACE;
    const uint32_t nb = (n + MLP_ROWS - 1) / MLP_ROWS;
    hipStream_t s = static_cast<hipStream_t>(stream);
    float* part = static_cast<float*>(workspace);
    clear_stale_error();
    hipLaunchKernelGGL(mlp_backward_kernel, dim3(nb), dim3(MLP_ROWS), 0, s, params, norm, x, t, n, y, h1t, h2t, part);
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3((NP + 1 + 255) / 256), dim3(256), 0, s, part, nb, n, grad, loss);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SPMD_OK : hip_fail(e);
}

int spmd_mlp_adam(float* params, const float* grad, float* m, float* v, uint32_t step, float lr, float beta1,
                  float beta2, float eps, void* stream) {
    if (!params || !grad || !m || !v || step == 0) return SPMD_ERR_ARGS;
    const float c1 = 1.0f - powf(beta1, (float)step), c2 = 1.0f - powf(beta2, (float)step);
    clear_stale_error();
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((NP + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(stream),
                       params, grad, m, v, lr, beta1, beta2, eps, c1, c2);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SPMD_OK : hip_fail(e);
}

int spmd_mlp_choose_batch(const float* params, uint32_t k_models, const float* norm, const float* feats,
                          uint32_t m, const float* cands, uint32_t c, const uint8_t* valid, const uint32_t* chunks,
                          float slack, uint32_t* best, float* best_pred, float* best_sd, void* stream) {
    if (!chunks || !(slack >= 0.0f) || !(slack < 1e30f)) return SPMD_ERR_ARGS;
    return choose_impl(params, k_models, norm, feats, m, cands, c, valid, chunks, log1pf(slack), best, best_pred,
                       best_sd, stream);
}

int spmd_mlp_choose(const float* params, uint32_t k_models, const float* norm, const float* feats, uint32_t m,
                    const float* cands, uint32_t c, const uint8_t* valid, uint32_t* best, float* best_pred,
                    float* best_sd, void* stream) {
    return choose_impl(params, k_models, norm, feats, m, cands, c, valid, nullptr, 0.0f, best, best_pred, best_sd,
                       stream);
}

}  // extern "C"

namespace {

int choose_impl(const float* params, uint32_t k_models, const float* norm, const float* feats, uint32_t m,
                const float* cands, uint32_t c, const uint8_t* valid, const uint32_t* chunks, float log_slack,
                uint32_t* best, float* best_pred, float* best_sd, void* stream) {
    if (!params || !norm || k_models == 0 || k_models > SPMD_MLP_MAX_MODELS) return SPMD_ERR_ARGS;
    if (c == 0 || c > SPMD_MLP_MAX_CANDS || !cands) return SPMD_ERR_ARGS;
    if (m && (!feats || !valid || !best || !best_pred || !best_sd)) return SPMD_ERR_ARGS;
    if (!m) return SPMD_OK;
    const size_t shm = (size_t)k_models * NP * sizeof(float);
    if (shm > 65536) {  // up to 4 models: 81 KB of the 160 KB LDS, opted in explicitly
        hipError_t ea = hipFuncSetAttribute(reinterpret_cast<const void*>(&mlp_choose_kernel),
                                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (ea != hipSuccess) return hip_fail(ea);
    }
    const uint32_t grid = m < 1024 ? m : 1024;
    clear_stale_error();
    hipLaunchKernelGGL(mlp_choose_kernel, dim3(grid), dim3(SPMD_MLP_MAX_CANDS), shm, static_cast<hipStream_t>(stream),
                       params, k_models, norm, feats, m, cands, c, valid, chunks, log_slack, best, best_pred,
                       best_sd);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SPMD_OK : hip_fail(e);
}

}  // namespace
