// cls_jacobi.hpp -- block body of the JACOBI5_F32 class: one sweep of the
// 5-point Laplace-Jacobi stencil.
//
// A BX x BY block owns a tile of BX columns and BY*C rows (each thread
// computes C cells down its column, C rows apart).  Phase 1 copies the tile
// and a one-cell halo from HBM into LDS; barrier; phase 2 computes every
// owned interior cell as 0.25f * ((N + S) + (W + E)) with each operation
// rounded to fp32 in that order (no contraction), and copies border cells.
// Cells outside the grid are neither loaded nor stored.
#pragma once
#include "common.hpp"

namespace spmd {

template <int BX, int BY, int C>
struct JacobiLds {
    float t[BY * C + 2][BX + 2];
};

template <int BX, int BY, int C>
__device__ __forceinline__ void jacobi_block(const float* __restrict__ u, float* __restrict__ v, uint32_t nx,
                                             uint32_t ny, uint32_t bx, uint32_t by, JacobiLds<BX, BY, C>& L) {
#pragma clang fp contract(off)
    constexpr int TY = BY * C;
    constexpr int H = TY + 2, W = BX + 2;
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int64_t x0 = (int64_t)bx * BX, y0 = (int64_t)by * TY;
    for (int r = ty; r < H; r += BY) {
        const int64_t gy = y0 - 1 + r;
        if (gy < 0 || gy >= (int64_t)ny) continue;
        const float* row = u + gy * (int64_t)nx;
        for (int cc = tx; cc < W; cc += BX) {
            const int64_t gx = x0 - 1 + cc;
            if (gx >= 0 && gx < (int64_t)nx) L.t[r][cc] = row[gx];
        }
    }
    __syncthreads();
    const int64_t gx = x0 + tx;
    if (gx >= (int64_t)nx) return;
    const bool xborder = (gx == 0) || (gx == (int64_t)nx - 1);
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const int r = ty + k * BY;
        const int64_t gy = y0 + r;
        if (gy >= (int64_t)ny) break;
        const float c = L.t[r + 1][tx + 1];
        float out;
        if (xborder || gy == 0 || gy == (int64_t)ny - 1) {
            out = c;
        } else {
            const float ns = L.t[r][tx + 1] + L.t[r + 2][tx + 1];
            const float we = L.t[r + 1][tx] + L.t[r + 1][tx + 2];
            const float sum = ns + we;
            out = 0.25f * sum;
        }
        v[gy * (int64_t)nx + gx] = out;
    }
}

}  // namespace spmd
