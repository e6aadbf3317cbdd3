// cls_gemm.hpp -- block body of the GEMM_F32 class: C = A * B, fp32
// row-major, fp32 accumulation on the matrix cores.
//
// A block of 256 threads (4 waves, 2 x 2) owns a T x T tile of C; each wave
// owns a (T/2) x (T/2) sub-tile made of (T/64)^2 tiles of 32 x 32, each
// accumulated by v_mfma_f32_32x32x2f32 (A fragment 32 x 2, B fragment
// 2 x 32, 16 fp32 accumulators per lane).  K is walked in KT = 16 deep
// slices staged in LDS: A transposed (k-major) so that the 32 lanes that
// need one k read 32 consecutive words, B as is.  The LDS has 64 banks of
// 4 bytes and serves a whole wave per access; an MFMA operand read takes
// k-rows kk (lanes 0-31) and kk + 1 (lanes 32-63), 4 banks apart with the
// 4-word row pad, so 28 of their banks collide.  At T = 256 odd k-rows are
// stored rotated by 28 columns (mod T): the two halves then land 32 banks
// apart, the transposed stores of A stay conflict-free, and the kernel
// gains 3.7%.  At T = 64 and 128 the rotation costs more in address
// arithmetic and lost paired reads than the conflicts do, so those tiles
// keep the plain layout.  Two LDS buffers and a register prefetch of the
// next slice let one barrier per slice separate the writers of one buffer
// from the readers of the other.  Outside the matrices the staged values
// are zero.  At T >= 128 a wave raises its issue priority for the MFMA
// part of each slice and drops it for the LDS stores and the barrier, so
// waves that can feed the matrix cores go first (tile 128: 1110 -> 1029 us
// at 4096^3; at T = 64 it measured no better).
//
// Operand layouts of v_mfma_f32_32x32x2f32 (64 lanes):
//   A: lane l holds A[m = l % 32][k = l / 32]
//   B: lane l holds B[k = l / 32][n = l % 32]
//   D: lane l, register r holds D[m = 8*(r/4) + 4*(l/32) + r%4][n = l % 32]
#pragma once
#include "common.hpp"
#include "warp32.hpp"

namespace spmd {

typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int GEMM_KT = 16;
constexpr int GEMM_PAD = 4;

// Physical column of logical column c in k-row k of a T-wide LDS slice.
template <int T>
__device__ __forceinline__ int gemm_lds_col(int k, int c) {
    if constexpr (T < 256) return c;
    else return (k & 1) ? ((c + 28) & (T - 1)) : c;
}

template <int T>
struct GemmLds {
    alignas(16) float a[2][GEMM_KT][T + GEMM_PAD];
    alignas(16) float b[2][GEMM_KT][T + GEMM_PAD];
};

template <int T>
__device__ __forceinline__ void gemm_block(const float* __restrict__ A, const float* __restrict__ B,
                                           float* __restrict__ C, uint32_t M, uint32_t N, uint32_t K, uint32_t bx,
                                           uint32_t by, bool vecA, bool vecB, GemmLds<T>& L) {
    constexpr int KT = GEMM_KT;
    constexpr int RT = T / 64;           // 32 x 32 tiles per wave edge
    constexpr int WT = T / 2;            // wave tile edge
    constexpr int PT = T * KT / 1024;    // float4 loads per thread per operand
    constexpr int KQ = KT / 4;           // float4 per row of an A slice
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t m0 = (int64_t)by * T, n0 = (int64_t)bx * T;
    const int64_t Mi = M, Ni = N, Ki = K;

    f32x16 acc[RT][RT];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < RT; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

    f32x4 ra[PT], rb[PT];
    // Interior slices (the whole T x KT and KT x T slices inside the
    // matrices, rows 16-byte aligned) are decided once per block and slice,
    // so their loads issue back to back with no per-thread branches; edge
    // slices take the element-wise path.
    const bool inner_mn = vecA && vecB && m0 + T <= Mi && n0 + T <= Ni;
    auto gload = [&](int kt) {
        const int64_t k0 = (int64_t)kt * KT;
        if (inner_mn && k0 + KT <= Ki) {
#pragma unroll
            for (int j = 0; j < PT; ++j) {
                const int q = tid + 256 * j;
                ra[j] = *reinterpret_cast<const f32x4*>(A + (m0 + q / KQ) * Ki + k0 + (q % KQ) * 4);
            }
#pragma unroll
            for (int j = 0; j < PT; ++j) {
                const int q = tid + 256 * j;
                rb[j] = *reinterpret_cast<const f32x4*>(B + (k0 + q / (T / 4)) * Ni + n0 + (q % (T / 4)) * 4);
            }
            return;
        }
#pragma unroll
        for (int j = 0; j < PT; ++j) {
            const int q = tid + 256 * j;  // A slice: T rows x KT/4 float4
            const int row = q / KQ, kq = (q % KQ) * 4;
            const int64_t gm = m0 + row, gk = k0 + kq;
#pragma unroll
            for (int e = 0; e < 4; ++e) ra[j][e] = (gm < Mi && gk + e < Ki) ? A[gm * Ki + gk + e] : 0.0f;
        }
#pragma unroll
        for (int j = 0; j < PT; ++j) {
            const int q = tid + 256 * j;  // B slice: KT rows x T/4 float4
            const int row = q / (T / 4), c4 = (q % (T / 4)) * 4;
            const int64_t gk = k0 + row, gn = n0 + c4;
#pragma unroll
            for (int e = 0; e < 4; ++e) rb[j][e] = (gk < Ki && gn + e < Ni) ? B[gk * Ni + gn + e] : 0.0f;
        }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int j = 0; j < PT; ++j) {
            const int q = tid + 256 * j;
            const int row = q / KQ, kq = (q % KQ) * 4;
#pragma unroll
            for (int e = 0; e < 4; ++e) L.a[buf][kq + e][gemm_lds_col<T>(kq + e, row)] = ra[j][e];
        }
#pragma unroll
        for (int j = 0; j < PT; ++j) {
            const int q = tid + 256 * j;
            const int row = q / (T / 4), c4 = (q % (T / 4)) * 4;
            *reinterpret_cast<f32x4*>(&L.b[buf][row][gemm_lds_col<T>(row, c4)]) = rb[j];
        }
    };

    const int nk = (int)((Ki + KT - 1) / KT);
    gload(0);
    lstore(0);
    __syncthreads();
    const int kl = lane >> 5, ml = lane & 31;
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) gload(kt + 1);
#pragma unroll
        for (int kk = 0; kk < KT; kk += 2) {
            float a[RT], b[RT];
#pragma unroll
            for (int i = 0; i < RT; ++i) a[i] = L.a[cur][kk + kl][gemm_lds_col<T>(kk + kl, wm * WT + i * 32 + ml)];
#pragma unroll
            for (int j = 0; j < RT; ++j) b[j] = L.b[cur][kk + kl][gemm_lds_col<T>(kk + kl, wn * WT + j * 32 + ml)];
            if constexpr (T >= 128) __builtin_amdgcn_s_setprio(1);
#pragma unroll
            for (int i = 0; i < RT; ++i)
#pragma unroll
                for (int j = 0; j < RT; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        if constexpr (T >= 128) __builtin_amdgcn_s_setprio(0);
        if (kt + 1 < nk) lstore(cur ^ 1);
        __syncthreads();
    }

#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < RT; ++j) {
            const int64_t col = n0 + wn * WT + j * 32 + ml;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t row = m0 + wm * WT + i * 32 + (r >> 2) * 8 + kl * 4 + (r & 3);
                if (row < Mi && col < Ni) C[row * Ni + col] = acc[i][j][r];
            }
        }
}

}  // namespace spmd
