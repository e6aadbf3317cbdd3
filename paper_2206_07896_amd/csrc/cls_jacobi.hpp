// cls_jacobi.hpp -- block body of the JACOBI5_F32 class: one sweep of the
// 5-point Laplace-Jacobi stencil.
//
// A BX x BY block owns a tile of BX columns and BY*C rows (each thread
// computes C cells down its column, BY rows apart).  Phase 1 copies the
// tile and a one-cell halo from HBM into LDS; barrier; phase 2 computes
// every owned interior cell as 0.25f * ((N + S) + (W + E)) with each
// operation rounded to fp32 in that order (no contraction), and copies
// border cells.  Cells outside the grid are never stored; halo cells
// outside the grid are staged as zero and never read.
#pragma once
#include "common.hpp"
#include "warp32.hpp"

namespace spmd {

template <int BX, int BY, int C>
struct JacobiLds {
    float t[BY * C + 2][BX + 2];
};

// A block's tile in three phases, so that a loop over blocks can issue one
// block's loads before it waits on the previous block's: every global load
// into registers, registers to the LDS tile (a barrier must follow), and
// the cells from the LDS tile.
// The interior columns take NP row passes per thread.  The two halo
// columns, 2H cells (H = BY*C + 2 rows), are spread over all threads: halo
// cell i = t + k*BX*BY is row i/2 of the west (i even) or east (i odd)
// column, NH = ceil(2H / threads) cells per thread (one for 64-wide blocks).
template <int BX, int BY, int C>
struct JacobiRegs {
    static constexpr int NP = (BY * C + 2 + BY - 1) / BY;          // row passes per thread
    static constexpr int NH = (2 * (BY * C + 2) + BX * BY - 1) / (BX * BY);  // halo cells per thread
    float vc[NP];                                                 // interior column
    float vh[NH];                                                 // halo cells
};

template <int BX, int BY, int C>
__device__ __forceinline__ void jacobi_load(const float* __restrict__ u, uint32_t nx, uint32_t ny, uint32_t bx,
                                            uint32_t by, int tx, int ty, JacobiRegs<BX, BY, C>& R) {
    constexpr int TY = BY * C;
    constexpr int H = TY + 2;
    constexpr int NP = JacobiRegs<BX, BY, C>::NP;
    constexpr int NH = JacobiRegs<BX, BY, C>::NH;
    const int64_t x0 = (int64_t)bx * BX, y0 = (int64_t)by * TY;
    const int64_t NX = nx, NY = ny;
    const int64_t gxc = x0 + tx;  // interior column of this thread
    const bool has_c = gxc < NX;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int r = ty + p * BY;
        const int64_t gy = y0 - 1 + r;
        const bool rowok = r < H && gy >= 0 && gy < NY;
        R.vc[p] = (rowok && has_c) ? u[gy * NX + gxc] : 0.0f;
    }
    const int t = ty * BX + tx;
#pragma unroll
    for (int k = 0; k < NH; ++k) {
        const int i = t + k * BX * BY;
        const int64_t gxh = (i & 1) ? x0 + BX : x0 - 1;  // west (i even) or east column
        const int64_t gyh = y0 - 1 + (i >> 1);
        const bool has_h = i < 2 * H && gxh >= 0 && gxh < NX && gyh >= 0 && gyh < NY;
        R.vh[k] = has_h ? u[gyh * NX + gxh] : 0.0f;
    }
}

template <int BX, int BY, int C>
__device__ __forceinline__ void jacobi_commit(int tx, int ty, const JacobiRegs<BX, BY, C>& R,
                                              JacobiLds<BX, BY, C>& L) {
    constexpr int H = BY * C + 2;
#pragma unroll
    for (int p = 0; p < JacobiRegs<BX, BY, C>::NP; ++p) {
        const int r = ty + p * BY;
        if (r < H) L.t[r][tx + 1] = R.vc[p];
    }
    const int t = ty * BX + tx;
#pragma unroll
    for (int k = 0; k < JacobiRegs<BX, BY, C>::NH; ++k) {
        const int i = t + k * BX * BY;
        if (i < 2 * H) L.t[i >> 1][(i & 1) ? BX + 1 : 0] = R.vh[k];
    }
}

template <int BX, int BY, int C>
__device__ __forceinline__ void jacobi_compute(float* __restrict__ v, uint32_t nx, uint32_t ny, uint32_t bx,
                                               uint32_t by, int tx, int ty, const JacobiLds<BX, BY, C>& L) {
#pragma clang fp contract(off)
    constexpr int TY = BY * C;
    const int64_t x0 = (int64_t)bx * BX, y0 = (int64_t)by * TY;
    const int64_t NX = nx, NY = ny;
    const int64_t gx = x0 + tx;
    if (gx >= NX) return;
    const bool xborder = (gx == 0) || (gx == NX - 1);
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const int r = ty + k * BY;
        const int64_t gy = y0 + r;
        if (gy >= NY) break;
        const float c = L.t[r + 1][tx + 1];
        float out;
        if (xborder || gy == 0 || gy == NY - 1) {
            out = c;
        } else {
            const float ns = L.t[r][tx + 1] + L.t[r + 2][tx + 1];
            const float we = L.t[r + 1][tx] + L.t[r + 1][tx + 2];
            const float sum = ns + we;
            out = 0.25f * sum;
        }
        v[gy * NX + gx] = out;
    }
}

// One block: every load of the tile and its halo is issued before the
// first LDS store, so each thread keeps NP (+1 halo) loads in flight.
template <int BX, int BY, int C>
__device__ __forceinline__ void jacobi_block(const float* __restrict__ u, float* __restrict__ v, uint32_t nx,
                                             uint32_t ny, uint32_t bx, uint32_t by, int tx, int ty,
                                             JacobiLds<BX, BY, C>& L) {
    JacobiRegs<BX, BY, C> R;
    jacobi_load<BX, BY, C>(u, nx, ny, bx, by, tx, ty, R);
    jacobi_commit<BX, BY, C>(tx, ty, R, L);
    __syncthreads();
    jacobi_compute<BX, BY, C>(v, nx, ny, bx, by, tx, ty, L);
}


// Workgroups are dealt to the 8 XCDs round-robin by linear id, and each XCD
// has its own L2.  Tile t of XCD x = id mod 8 is the (id / 8)-th of a
// contiguous range of tiles, so neighbouring tiles -- which read each
// other's edge lines as halo -- run on the same XCD and share its L2.
constexpr uint32_t NUM_XCD = 8;

__device__ __forceinline__ uint32_t xcd_tile(uint32_t id, uint32_t nt) {
    const uint32_t q = nt / NUM_XCD, r = nt % NUM_XCD;
    const uint32_t x = id % NUM_XCD, local = id / NUM_XCD;
    return x < r ? x * (q + 1) + local : r * (q + 1) + (x - r) * q + local;
}

// Vector form, for nx a multiple of 4 and 16-byte aligned rows: a workgroup
// of 64 x BY threads owns 256 columns and BY*C rows, each thread four
// consecutive columns (one 16-byte load or store per row) and C rows, BY
// rows apart.  The interior sits at LDS column 4 so that every row of four
// is 16-byte aligned; the halo columns sit at 3 and 260.  Each cell is
// computed exactly as in jacobi_block.
constexpr int JV_W = 256, JV_LD = JV_W + 8;

template <int BY, int C>
struct JacobiV4Lds {
    alignas(16) float t[BY * C + 2][JV_LD];
};

template <int BY, int C>
__device__ __forceinline__ void jacobi_block_v4(const float* __restrict__ u, float* __restrict__ v, uint32_t nx,
                                                uint32_t ny, uint32_t bx, uint32_t by, int tx, int ty,
                                                JacobiV4Lds<BY, C>& L) {
#pragma clang fp contract(off)
    constexpr int TY = BY * C;
    constexpr int H = TY + 2;
    constexpr int NP = (H + BY - 1) / BY;
    const int64_t x0 = (int64_t)bx * JV_W, y0 = (int64_t)by * TY;
    const int64_t NX = nx, NY = ny;
    const int64_t gx0 = x0 + 4 * tx;                 // first of this thread's four columns
    const int64_t gxh = tx == 0 ? x0 - 1 : x0 + JV_W;  // halo column (threads tx < 2)
    const bool has_c = gx0 < NX;                     // then all four are (NX % 4 == 0)
    const bool has_h = tx < 2 && gxh >= 0 && gxh < NX;
    f32x4 vc[NP];
    float vh[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int r = ty + p * BY;
        const int64_t gy = y0 - 1 + r;
        const bool rowok = r < H && gy >= 0 && gy < NY;
        const f32x4 z = {0.0f, 0.0f, 0.0f, 0.0f};
        vc[p] = (rowok && has_c) ? *reinterpret_cast<const f32x4*>(u + gy * NX + gx0) : z;
        vh[p] = (rowok && has_h) ? u[gy * NX + gxh] : 0.0f;
    }
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int r = ty + p * BY;
        if (r < H) {
            *reinterpret_cast<f32x4*>(&L.t[r][4 + 4 * tx]) = vc[p];
            if (tx < 2) L.t[r][tx == 0 ? 3 : 4 + JV_W] = vh[p];
        }
    }
    __syncthreads();
    if (!has_c) return;
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const int r = ty + k * BY;
        const int64_t gy = y0 + r;
        if (gy >= NY) break;
        const f32x4 c = *reinterpret_cast<const f32x4*>(&L.t[r + 1][4 + 4 * tx]);
        f32x4 out = c;
        if (gy != 0 && gy != NY - 1) {
            const f32x4 n = *reinterpret_cast<const f32x4*>(&L.t[r][4 + 4 * tx]);
            const f32x4 s = *reinterpret_cast<const f32x4*>(&L.t[r + 2][4 + 4 * tx]);
            const float wl = L.t[r + 1][3 + 4 * tx];
            const float er = L.t[r + 1][8 + 4 * tx];
            const float w[4] = {wl, c.x, c.y, c.z};
            const float e[4] = {c.y, c.z, c.w, er};
            const float nn[4] = {n.x, n.y, n.z, n.w};
            const float ss[4] = {s.x, s.y, s.z, s.w};
            const float cc[4] = {c.x, c.y, c.z, c.w};
            float o[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t gx = gx0 + j;
                if (gx == 0 || gx == NX - 1) {
                    o[j] = cc[j];
                } else {
                    const float ns = nn[j] + ss[j];
                    const float we = w[j] + e[j];
                    const float sum = ns + we;
                    o[j] = 0.25f * sum;
                }
            }
            out.x = o[0];
            out.y = o[1];
            out.z = o[2];
            out.w = o[3];
        }
        // Nontemporal: no part of this sweep reads v again.  Whole-line
        // 16-byte stores gain from it (92.5 -> 88.5 us per 8192^2 sweep);
        // the 4-byte stores of the general-width body lost 4% on the mixed
        // queue with it, so they stay plain.
        __builtin_nontemporal_store(out, reinterpret_cast<f32x4*>(v + gy * NX + gx0));
    }
}

// General-width form, for any nx and alignment: a workgroup of 64 x BY
// threads owns 256 columns and BY*C rows; thread tx holds columns tx,
// tx + 64, tx + 128 and tx + 192 of the tile (a wave's four loads of one row
// cover 1 KiB contiguous) and C rows, BY rows apart.  The interior sits at
// LDS columns 1..256, the halo at 0 and 257; the halo cells are spread over
// all threads.  Each cell is computed exactly as in jacobi_block.
constexpr int JW_LD = JV_W + 2;

template <int BY, int C>
struct JacobiWLds {
    float t[BY * C + 2][JW_LD];
};

template <int BY, int C>
__device__ __forceinline__ void jacobi_block_w(const float* __restrict__ u, float* __restrict__ v, uint32_t nx,
                                               uint32_t ny, uint32_t bx, uint32_t by, int tx, int ty,
                                               JacobiWLds<BY, C>& L) {
#pragma clang fp contract(off)
    constexpr int TY = BY * C;
    constexpr int H = TY + 2;
    constexpr int NP = (H + BY - 1) / BY;
    constexpr int T = 64 * BY;
    constexpr int NH = (2 * H + T - 1) / T;
    const int64_t x0 = (int64_t)bx * JV_W, y0 = (int64_t)by * TY;
    const int64_t NX = nx, NY = ny;
    float vc[NP][4], vh[NH];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int r = ty + p * BY;
        const int64_t gy = y0 - 1 + r;
        const bool rowok = r < H && gy >= 0 && gy < NY;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t gx = x0 + tx + 64 * q;
            vc[p][q] = (rowok && gx < NX) ? u[gy * NX + gx] : 0.0f;
        }
    }
    const int t = ty * 64 + tx;
#pragma unroll
    for (int k = 0; k < NH; ++k) {
        const int i = t + k * T;
        const int64_t gxh = (i & 1) ? x0 + JV_W : x0 - 1;  // east (i odd) or west column
        const int64_t gyh = y0 - 1 + (i >> 1);
        const bool has_h = i < 2 * H && gxh >= 0 && gxh < NX && gyh >= 0 && gyh < NY;
        vh[k] = has_h ? u[gyh * NX + gxh] : 0.0f;
    }
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int r = ty + p * BY;
        if (r < H) {
#pragma unroll
            for (int q = 0; q < 4; ++q) L.t[r][1 + tx + 64 * q] = vc[p][q];
        }
    }
#pragma unroll
    for (int k = 0; k < NH; ++k) {
        const int i = t + k * T;
        if (i < 2 * H) L.t[i >> 1][(i & 1) ? JV_W + 1 : 0] = vh[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const int r = ty + k * BY;
        const int64_t gy = y0 + r;
        if (gy >= NY) break;
        const bool yborder = gy == 0 || gy == NY - 1;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t gx = x0 + tx + 64 * q;
            if (gx >= NX) break;
            const int lx = 1 + tx + 64 * q;
            const float c = L.t[r + 1][lx];
            float out;
            if (yborder || gx == 0 || gx == NX - 1) {
                out = c;
            } else {
                const float ns = L.t[r][lx] + L.t[r + 2][lx];
                const float we = L.t[r + 1][lx - 1] + L.t[r + 1][lx + 1];
                const float sum = ns + we;
                out = 0.25f * sum;
            }
            v[gy * NX + gx] = out;
        }
    }
}

}  // namespace spmd
