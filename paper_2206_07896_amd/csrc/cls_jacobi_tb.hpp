// cls_jacobi_tb.hpp -- block body of the JACOBI5T_F32 class: S sweeps of the
// 5-point Laplace-Jacobi stencil in one pass over HBM (temporal blocking).
//
// One sweep reads and writes every cell once, so a sweep-per-launch stencil
// is bound at 8 bytes per cell by HBM.  Here a workgroup loads a region of
// 256 columns x (64 + 2H) rows -- its (256 - 2H) x 64 interior tile and an
// H-cell halo, H >= S -- runs S sweeps on it, and writes back only the
// interior: HBM moves about 8 bytes per cell per S sweeps, plus the halo.
//
// The region lives in registers.  A wave spans a whole region row (64
// lanes x 4 columns); the 4 waves own bands of RS = (64 + 2H) / 4
// consecutive rows, each lane its 4 columns of every row of its band.  In a
// sweep, north and south neighbours come from the lane's own registers, west
// and east from the adjacent lanes (a full-wave shuffle), and only the first
// and last row of each band go through LDS to the neighbouring waves (two
// slots per sweep parity, one barrier per sweep).
//
// Phases:
//   load   the region row by row, 16 bytes per lane; cells outside the grid
//          are zero (a cell that is updated never reads them);
//   sweep  S times: publish the band's edge rows; barrier; read the
//          neighbours' edge rows; update the band top-down.  A cell is
//          updated as 0.25f * ((N + S) + (W + E)), each operation rounded
//          to fp32 in that order (no contraction), exactly as the one-sweep
//          class; border cells of the grid keep their value.  Sweep s only
//          needs region rows [s, 64 + 2H - s), so the others are skipped;
//          the region's outer columns go stale one per sweep (their outer
//          neighbours do not exist), and after S sweeps the stale ring is
//          still outside the interior (H >= S);
//   store  the interior, cells inside the grid.
// Results are bit-identical to S sweeps of the one-sweep class.
#pragma once
#include "cls_jacobi.hpp"

namespace spmd {

constexpr int JT_H = 64, JT_THREADS = 256, JT_WAVES = JT_THREADS / 64;

// interior tile width for halo H
__host__ __device__ constexpr int jt_width(int h) { return 256 - 2 * h; }

struct JacobiTbLds {
    f32x4 edge[2][2][JT_WAVES][64];  // [sweep parity][first row, last row][wave][lane]
};

template <int H>
__device__ __forceinline__ void jacobi_tb_block(const float* __restrict__ u, float* __restrict__ v, uint32_t nx,
                                                uint32_t ny, uint32_t sweeps, uint32_t bx, uint32_t by,
                                                JacobiTbLds& L) {
#pragma clang fp contract(off)
    constexpr int ROWS = JT_H + 2 * H;
    constexpr int RS = ROWS / JT_WAVES;
    static_assert(ROWS % JT_WAVES == 0 && H % 4 == 0, "bands of whole rows, 16-byte groups");
    const int lane = (int)(threadIdx.x & 63u), w = (int)(threadIdx.x >> 6);
    const int64_t NX = nx, NY = ny;
    const int64_t x0 = (int64_t)bx * jt_width(H) - H, y0 = (int64_t)by * JT_H - H;  // region origin
    const int64_t gx = x0 + 4 * lane;  // this lane's first column
    const int r0 = w * RS;             // this wave's first region row
    const f32x4 z = {0.0f, 0.0f, 0.0f, 0.0f};

    f32x4 c[RS];
    const bool col_in = gx >= 0 && gx < NX;  // all four columns (NX % 4 == 0)
#pragma unroll
    for (int i = 0; i < RS; ++i) {
        const int64_t gy = y0 + r0 + i;
        c[i] = (col_in && gy >= 0 && gy < NY) ? __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(u + gy * NX + gx))
                                              : z;
    }
    bool col_upd[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) col_upd[j] = gx + j >= 1 && gx + j <= NX - 2;

    for (int s = 1; s <= (int)sweeps; ++s) {
        const int par = s & 1;
        L.edge[par][0][w][lane] = c[0];
        L.edge[par][1][w][lane] = c[RS - 1];
        __syncthreads();
        const f32x4 up = w > 0 ? L.edge[par][1][w - 1][lane] : z;
        const f32x4 dn = w < JT_WAVES - 1 ? L.edge[par][0][w + 1][lane] : z;
        f32x4 prev = up;  // this sweep's input of the row above
#pragma unroll
        for (int i = 0; i < RS; ++i) {
            const int r = r0 + i;
            const f32x4 cur = c[i];
            const f32x4 below = i + 1 < RS ? c[i + 1] : dn;
            if (r >= s && r < ROWS - s) {  // wave-uniform
                const float wl = __shfl_up(cur.w, 1u);
                const float er = __shfl_down(cur.x, 1u);
                const int64_t gy = y0 + r;
                if (gy >= 1 && gy <= NY - 2) {  // wave-uniform
                    const float ww[4] = {wl, cur.x, cur.y, cur.z};
                    const float ee[4] = {cur.y, cur.z, cur.w, er};
                    const float nn[4] = {prev.x, prev.y, prev.z, prev.w};
                    const float ss[4] = {below.x, below.y, below.z, below.w};
                    const float cc[4] = {cur.x, cur.y, cur.z, cur.w};
                    float o[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const float ns = nn[j] + ss[j];
                        const float we = ww[j] + ee[j];
                        const float sum = ns + we;
                        o[j] = col_upd[j] ? 0.25f * sum : cc[j];
                    }
                    c[i].x = o[0];
                    c[i].y = o[1];
                    c[i].z = o[2];
                    c[i].w = o[3];
                }
            }
            prev = cur;
        }
    }

    if (lane >= H / 4 && lane < 64 - H / 4 && gx < NX) {
#pragma unroll
        for (int i = 0; i < RS; ++i) {
            const int r = r0 + i;
            const int64_t gy = y0 + r;
            if (r >= H && r < H + JT_H && gy < NY) *reinterpret_cast<f32x4*>(v + gy * NX + gx) = c[i];
        }
    }
}

}  // namespace spmd
