// synth_fill.hip -- device-side seeded input generator (spmd_synth.h).
// Input generation only; it shares no code with the kernel classes.
#include "common.hpp"
#include "spmd_synth.h"

namespace spmd {

constexpr uint64_t SM_GAMMA = 0x9E3779B97F4A7C15ull;

__host__ __device__ __forceinline__ uint64_t sm_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

enum { FILL_I32 = 0, FILL_F32 = 1, FILL_RAW = 2, FILL_ZIPF = 3 };

__global__ __launch_bounds__(256) void synth_fill_kernel(int kind, void* out, uint64_t count, uint64_t key,
                                                         uint64_t start, int32_t lo, uint64_t span,
                                                         const double* cdf, uint32_t k) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        const uint64_t h = sm_mix(key + (start + i + 1) * SM_GAMMA);
        switch (kind) {
        case FILL_I32:
            static_cast<int32_t*>(out)[i] = (int32_t)((int64_t)lo + (int64_t)(((h >> 32) * span) >> 32));
            break;
        case FILL_F32: static_cast<float*>(out)[i] = (float)(h >> 40) * 0x1.0p-24f; break;
        case FILL_RAW: static_cast<uint32_t*>(out)[i] = (uint32_t)(h >> 32); break;
        default: {
            const double u = (double)(h >> 11) * 0x1.0p-53;
            uint32_t a = 0, b = k;  // first index with cdf[idx] > u
            while (a < b) {
                const uint32_t m = (a + b) >> 1;
                if (cdf[m] <= u) a = m + 1;
                else b = m;
            }
            static_cast<uint32_t*>(out)[i] = a < k ? a : k - 1;
        }
        }
    }
}

static int fill(int kind, void* out, uint64_t count, uint64_t seed, uint64_t start, int32_t lo, uint64_t span,
                const double* cdf, uint32_t k, void* stream) {
    if (!count) return SPMD_OK;
    if (!out) return SPMD_ERR_ARGS;
    const uint64_t blocks = (count + 255) / 256;
    const uint32_t g = (uint32_t)(blocks < 16384 ? blocks : 16384);
    clear_stale_error();
    hipLaunchKernelGGL(synth_fill_kernel, dim3(g), dim3(256), 0, static_cast<hipStream_t>(stream), kind, out, count,
                       sm_mix(seed), start, lo, span, cdf, k);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SPMD_OK : hip_fail(e);
}

}  // namespace spmd

using namespace spmd;

extern "C" {

uint64_t spmd_synth_key(uint64_t seed) { return sm_mix(seed); }

int spmd_synth_uniform_i32(int32_t* out, uint64_t count, uint64_t seed, uint64_t start, int32_t lo, int32_t hi,
                           void* stream) {
    if (hi < lo) return SPMD_ERR_ARGS;
    return fill(FILL_I32, out, count, seed, start, lo, (uint64_t)((int64_t)hi - (int64_t)lo + 1), nullptr, 0, stream);
}

int spmd_synth_uniform_f32(float* out, uint64_t count, uint64_t seed, uint64_t start, void* stream) {
    return fill(FILL_F32, out, count, seed, start, 0, 0, nullptr, 0, stream);
}

int spmd_synth_raw_u32(uint32_t* out, uint64_t count, uint64_t seed, uint64_t start, void* stream) {
    return fill(FILL_RAW, out, count, seed, start, 0, 0, nullptr, 0, stream);
}

int spmd_synth_zipf_u32(uint32_t* out, uint64_t count, uint64_t seed, uint64_t start, const double* cdf, uint32_t k,
                        void* stream) {
    if (!cdf || k == 0 || k > 65536) return SPMD_ERR_ARGS;
    return fill(FILL_ZIPF, out, count, seed, start, 0, 0, cdf, k, stream);
}

}  // extern "C"
