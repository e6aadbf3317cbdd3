// cls_gemm.hpp -- block bodies of the GEMM_F32 class: C = A * B, fp32
// row-major, fp32 accumulation on the matrix cores.  Shapes with 16-byte
// rows (K and N multiples of 4, aligned bases) take the direct-to-LDS form
// at the end of this file; the register-staged form below serves the rest.
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
#include <type_traits>

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


// ---- Direct-to-LDS form (16-byte aligned rows: K % 4 == 0, N % 4 == 0) ----
//
// Each K slice (16 deep) goes from HBM to LDS with global_load_lds_dwordx4:
// a lane's 16 bytes land at the instruction's LDS base + 16 * lane, so no
// register holds the slice and no LDS store is issued, and NS slices are in
// flight at once (a stage each).  Both operands are laid out for that:
//   A as [m][k] (k contiguous, 64-byte rows); the four 16-byte chunks of
//     row m sit at positions c ^ ((m / 4) % 4), so the 16-lane groups of a
//     16-byte read hit 16 distinct 4-bank groups;
//   B as [k][n]; rows with bit 2 of k set are rotated by 32 columns, so the
//     two half-waves of a read (k and k + 4, same columns) are 32 banks
//     apart.
// The contraction order inside an 8-deep group of k is permuted: in MFMA
// step s, lanes 0-31 take k = 8g + s and lanes 32-63 take k = 8g + 4 + s,
// for A and B alike, so one 16-byte LDS read gives a lane its A values for
// four steps.  A wave waits for its own loads of a slice (vmcnt) and a
// barrier then makes every wave's loads of that slice visible; the stage
// freed by the previous slice is refilled right after that barrier.
// Rows of A past M and columns of B past N are read from the last row or
// column instead (their products land outside C and are not stored); a K
// tail shorter than a slice is loaded through registers with zero fill.
constexpr int GEMM_DMA_KT = 16;

typedef __attribute__((address_space(1))) void gemm_gvoid;
typedef __attribute__((address_space(3))) void gemm_lvoid;

// s_waitcnt: vmcnt <= n, lgkmcnt 0, expcnt not waited (n < 16)
#define GEMM_WAIT_VM(n) __builtin_amdgcn_s_waitcnt(0x70 | (n))

// The stages are separate LDS arrays passed in by the kernel: the
// compiler then tells a refill from the reads of another stage and does
// not wait for the refill before those reads.
template <int T, int NS>
__device__ __forceinline__ void gemm_block_dma(const float* __restrict__ A, const float* __restrict__ B,
                                               float* __restrict__ C, uint32_t M, uint32_t N, uint32_t K,
                                               uint32_t bx, uint32_t by, float* S0, float* S1, float* S2,
                                               float* S3) {
    constexpr int KT = GEMM_DMA_KT;
    constexpr int RT = T / 64, WT = T / 2;
    constexpr int CPR = KT / 4;          // 16-byte chunks per A row
    constexpr int RPS = 64 / KT;         // A rows per 64-bank span
    constexpr int NI = T * KT / 1024;    // loads per wave per operand per slice
    constexpr int LPW = 2 * NI;          // loads per wave per slice
    constexpr int BCH = T / 4;           // 16-byte chunks per B row
    constexpr int SA = T * KT;           // floats per operand per stage
    static_assert(NS >= 2 && NS <= 4 && LPW * (NS - 2) < 16, "stage count");
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t m0 = (int64_t)by * T, n0 = (int64_t)bx * T;
    const int64_t Mi = M, Ni = N, Ki = K;
    if (m0 >= Mi || n0 >= Ni) return;  // a block wholly outside C (grids may be larger)
    const int nk = (int)(Ki / KT);

    // Per-lane source offsets from the block's slice-0 corner (the launcher
    // checks T * K and KT * N against 2^31).
    const float* Ab = A + m0 * Ki;
    const float* Bb = B + n0;
    int srcA[NI], srcB[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int ci = 64 * (wave + 4 * i) + lane;
        const int r = ci / CPR, c = (ci % CPR) ^ ((r / RPS) % CPR);
        const int rr = m0 + r < Mi ? r : (int)(Mi - 1 - m0);  // past M: the last row
        srcA[i] = rr * (int)K + 4 * c;
        const int k = ci / BCH;
        const int col = (4 * (ci % BCH) - ((k & 4) ? 32 : 0) + T) % T;
        const int cc = n0 + col < Ni ? col : (int)(Ni - 4 - n0);  // past N: the last chunk
        srcB[i] = k * (int)N + cc;
    }
    auto issue = [&](int kt, float* st) {
        const float* a = Ab + (int64_t)kt * KT;
        const float* b = Bb + (int64_t)kt * KT * Ni;
#pragma unroll
        for (int i = 0; i < NI; ++i)
            __builtin_amdgcn_global_load_lds((gemm_gvoid*)(a + srcA[i]), (gemm_lvoid*)(st + 256 * (wave + 4 * i)), 16, 0, 0);
#pragma unroll
        for (int i = 0; i < NI; ++i)
            __builtin_amdgcn_global_load_lds((gemm_gvoid*)(b + srcB[i]), (gemm_lvoid*)(st + SA + 256 * (wave + 4 * i)),
                                             16, 0, 0);
    };

    f32x16 acc[RT][RT];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < RT; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

    const int kl = lane >> 5, ml = lane & 31;
    const int aswz = (ml / RPS) % CPR;  // rows wm*WT + 32 i + ml share it
    int bcol[RT];
#pragma unroll
    for (int j = 0; j < RT; ++j) bcol[j] = (wn * WT + 32 * j + ml + 32 * kl) % T;
    auto compute = [&](const float* st) {
        const float* as = st;
        const float* bs = st + SA;
#pragma unroll
        for (int g = 0; g < KT / 8; ++g) {
            f32x4 av[RT];
            float bv[RT][4];
#pragma unroll
            for (int i = 0; i < RT; ++i)
                av[i] = *reinterpret_cast<const f32x4*>(as + (wm * WT + 32 * i + ml) * KT + 4 * ((2 * g + kl) ^ aswz));
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int j = 0; j < RT; ++j) bv[j][s] = bs[(8 * g + 4 * kl + s) * T + bcol[j]];
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int i = 0; i < RT; ++i)
#pragma unroll
                    for (int j = 0; j < RT; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i][s], bv[j][s], acc[i][j], 0, 0, 0);
        }
    };
    // Wait until at most `inflight` of this wave's loads are outstanding and
    // its LDS reads are done, then barrier.  The empty asm statements keep
    // the compiler from moving LDS accesses across the barrier; unlike
    // __syncthreads they add no wait for every outstanding load.
    auto barrier_vm = [&](auto inflight) {
        GEMM_WAIT_VM(decltype(inflight)::value);
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
    };
    auto stage = [&](auto idx) -> float* {
        constexpr int i = decltype(idx)::value;
        if constexpr (i == 0) return S0;
        else if constexpr (i == 1) return S1;
        else if constexpr (i == 2) return S2;
        else return S3;
    };
    // Slice kt is in stage sc: wait for it, refill the stage freed by slice
    // kt - 1 with slice kt + NS - 1, compute.  Inside the main loop every
    // refill is in range, so the wait count holds on every path (a refill
    // that may be skipped would make the compiler wait for all loads).
    auto step = [&](int kt, auto cur, auto full) {
        constexpr int sc = decltype(cur)::value;
        constexpr int sn = (sc + NS - 1) % NS;
        if constexpr (decltype(full)::value) {
            barrier_vm(std::integral_constant<int, LPW * (NS - 2)>());
            issue(kt + NS - 1, stage(std::integral_constant<int, sn>()));
        } else {
            barrier_vm(std::integral_constant<int, 0>());
            if (kt + NS - 1 < nk) issue(kt + NS - 1, stage(std::integral_constant<int, sn>()));
        }
        compute(stage(std::integral_constant<int, sc>()));
    };
    using Full = std::true_type;
    using Tail = std::false_type;
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;
    if (nk > 0) {
        // Slices 0 .. NS - 2, unconditionally (clamped to slice 0), so every
        // path into the loop has the same loads in flight.
        issue(0, S0);
        if constexpr (NS > 2) issue(nk > 1 ? 1 : 0, S1);
        if constexpr (NS > 3) issue(nk > 2 ? 2 : 0, S2);
        int kt = 0;
        for (; kt + 2 * NS - 2 < nk; kt += NS) {
            step(kt, I0(), Full());
            step(kt + 1, I1(), Full());
            if constexpr (NS > 2) step(kt + 2, I2(), Full());
            if constexpr (NS > 3) step(kt + 3, I3(), Full());
        }
        // at most 2 NS - 2 slices remain, the first in stage 0
        if (kt < nk) step(kt, I0(), Tail());
        if (kt + 1 < nk) step(kt + 1, I1(), Tail());
        if constexpr (NS == 3) {
            if (kt + 2 < nk) step(kt + 2, I2(), Tail());
            if (kt + 3 < nk) step(kt + 3, I0(), Tail());
        } else if constexpr (NS == 4) {
            if (kt + 2 < nk) step(kt + 2, I2(), Tail());
            if (kt + 3 < nk) step(kt + 3, I3(), Tail());
            if (kt + 4 < nk) step(kt + 4, I0(), Tail());
            if (kt + 5 < nk) step(kt + 5, I1(), Tail());
        }
        GEMM_WAIT_VM(0);  // the clamped prologue loads too: nothing lands later
        __syncthreads();  // every wave is done reading the stages
    }
    if (Ki % KT) {
        // The K tail (4, 8 or 12 deep, since K % 4 == 0) through registers,
        // zero outside the matrices, into stage 0 in the same layouts.
        const int64_t k0 = (int64_t)nk * KT;
        for (int ci = tid; ci < T * CPR; ci += 256) {
            const int r = ci / CPR, c = ci % CPR;
            f32x4 v = {0.0f, 0.0f, 0.0f, 0.0f};
            if (m0 + r < Mi && k0 + 4 * c < Ki) v = *reinterpret_cast<const f32x4*>(A + (m0 + r) * Ki + k0 + 4 * c);
            *reinterpret_cast<f32x4*>(S0 + r * KT + 4 * (c ^ ((r / RPS) % CPR))) = v;
        }
        for (int ci = tid; ci < KT * BCH; ci += 256) {
            const int k = ci / BCH, col = 4 * (ci % BCH);
            f32x4 v = {0.0f, 0.0f, 0.0f, 0.0f};
            if (k0 + k < Ki && n0 + col < Ni) v = *reinterpret_cast<const f32x4*>(B + (k0 + k) * Ni + n0 + col);
            *reinterpret_cast<f32x4*>(S0 + SA + k * T + (col + ((k & 4) ? 32 : 0)) % T) = v;
        }
        __syncthreads();
        compute(S0);
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
