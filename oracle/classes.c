/* Oracle kernel-class programs (TEST INFRASTRUCTURE ONLY).
 *
 * Each class is written the way the paper's SPMD-to-MPMD transformation
 * leaves a CUDA kernel (Section III-B3): a block body that is a sequence of
 * thread loops, one per region between two __syncthreads, with warp-level
 * code as nested warp/lane loops split at every warp operation.  Private
 * variables that live across a barrier are replicated per thread
 * (register slots); block-uniform values (loop counters of loops that
 * contain barriers) live in the block driver.  Shared memory is the block's
 * poisoned array; the dynamic part starts at b->dyn_base (Section III-B1,
 * III-B2).  A host driver per class sets up the launch(es) the way the
 * host program would and runs them serially or on the thread pool
 * (Section IV).
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "mpmd.h"

#define U32(x) ((uint32_t)(x))

typedef struct {
    int pool;      /* 0: serial executor; >0: thread-pool runtime       */
    uint32_t bpf;  /* blocks per fetch on the pool (0 = average)         */
    ox_stats st;   /* filled by pool runs                                */
} run_opts;

static int launch(ox_launch *L, run_opts *o, char *msg) {
    if (o && o->pool > 0) {
        int rc = ox_pool_start(o->pool);
        if (rc) return rc;
        return ox_pool_run(L, o->bpf, &o->st, msg);
    }
    return ox_run(L, msg);
}

static void set_dims(ox_launch *L, uint32_t gx, uint32_t gy, uint32_t bx, uint32_t by) {
    L->grid[0] = gx;
    L->grid[1] = gy;
    L->grid[2] = 1;
    L->block[0] = bx;
    L->block[1] = by;
    L->block[2] = 1;
}

static int is_pow2(uint32_t v) { return v && !(v & (v - 1)); }

/* ===================================================================== */
/* REDUCE_I32: block tree reduction, one partial per block, the last      */
/* block to finish sums the partials.                                      */
/*   buffers: 0 x[n], 1 partials[G], 2 out[1], 3 ticket counter[1]        */
/*   shared:  static word 0 = "this block is last" flag; dynamic s[B]     */
/*   Block b owns x[b*S, min((b+1)*S, n)) with S = 4*ceil(n / (4*G)).     */
/* ===================================================================== */
typedef struct {
    uint32_t n;
    uint32_t seg;
    int skip_barrier; /* fault injection: merge two tree levels */
} reduce_params;

#define RD_S(t) (b->dyn_base + 4ull * (t))

static int rd_load(ox_block *b, uint32_t t) {
    const reduce_params *p = b->params;
    uint64_t lo = (uint64_t)b->bidx[0] * p->seg;
    uint64_t hi = lo + p->seg < p->n ? lo + p->seg : p->n;
    uint32_t acc = 0;
    for (uint64_t j = lo + t; j < hi; j += b->block[0]) acc += ox_g_ld32(b, 0, j);
    ox_s_st32(b, RD_S(t), acc);
    return 0;
}

/* one tree level: if t < stride, s[t] += s[t + stride] */
static int rd_level(ox_block *b, uint32_t t) {
    uint32_t stride = (uint32_t)b->u[0];
    if (t < stride) ox_s_st32(b, RD_S(t), ox_s_ld32(b, RD_S(t)) + ox_s_ld32(b, RD_S(t + stride)));
    return 0;
}

/* two tree levels without the barrier between them (planted race) */
static int rd_level_pair_racy(ox_block *b, uint32_t t) {
    uint32_t stride = (uint32_t)b->u[0];
    if (t < stride) ox_s_st32(b, RD_S(t), ox_s_ld32(b, RD_S(t)) + ox_s_ld32(b, RD_S(t + stride)));
    uint32_t s2 = stride / 2;
    if (t < s2) ox_s_st32(b, RD_S(t), ox_s_ld32(b, RD_S(t)) + ox_s_ld32(b, RD_S(t + s2)));
    return 0;
}

/* thread 0: publish the partial, take a completion ticket (after a fence
 * in CUDA), record whether this block finished last */
static int rd_publish(ox_block *b, uint32_t t) {
    if (t == 0) {
        ox_g_st32(b, 1, b->bidx[0], ox_s_ld32(b, RD_S(0)));
        uint32_t ticket = ox_g_atomic_add32(b, 3, 0, 1u);
        ox_s_st32(b, 0, ticket == b->grid[0] - 1u);
    }
    return 0;
}

static int rd_final_load(ox_block *b, uint32_t t) {
    uint32_t last = ox_s_ld32(b, 0);
    if (last) {
        uint32_t acc = 0;
        for (uint64_t j = t; j < b->grid[0]; j += b->block[0]) acc += ox_g_ld32(b, 1, j);
        ox_s_st32(b, RD_S(t), acc);
    }
    return (int)last;
}

static int rd_final_level(ox_block *b, uint32_t t) {
    uint32_t last = ox_s_ld32(b, 0);
    if (last) rd_level(b, t);
    return (int)last;
}

static int rd_final_write(ox_block *b, uint32_t t) {
    uint32_t last = ox_s_ld32(b, 0);
    if (last && t == 0) {
        ox_g_st32(b, 2, 0, ox_s_ld32(b, RD_S(0)));
        ox_g_st32(b, 3, 0, 0u); /* leave the counter ready for the next launch */
    }
    return (int)last;
}

static void reduce_body(ox_block *b) {
    const reduce_params *p = b->params;
    uint32_t B = b->block[0];
    ox_threads(b, rd_load);
    int skipped = 0;
    for (uint32_t stride = B / 2; stride >= 1; stride /= 2) {
        b->u[0] = stride;
        if (p->skip_barrier && !skipped && stride >= 2 && stride <= 64) {
            ox_threads(b, rd_level_pair_racy);
            stride /= 2;
            skipped = 1;
            continue;
        }
        ox_threads(b, rd_level);
    }
    ox_threads(b, rd_publish);
    ox_threads(b, rd_final_load);
    for (uint32_t stride = B / 2; stride >= 1; stride /= 2) {
        b->u[0] = stride;
        ox_threads(b, rd_final_level);
    }
    ox_threads(b, rd_final_write);
}

int oracle_reduce_i32(const int32_t *x, uint32_t n, uint32_t grid, uint32_t block, int32_t *partials,
                      int32_t *out, uint64_t order_seed, int pool, uint32_t bpf, int skip_barrier,
                      char *msg) {
    if (grid == 0 || !is_pow2(block) || block < 32 || block > 1024) {
        snprintf(msg, 192, "reduce: bad launch shape");
        return OX_ERR_CONFIG;
    }
    reduce_params p = {n, 4u * (U32((n + 4ull * grid - 1) / (4ull * grid))), skip_barrier};
    uint32_t counter = 0;
    ox_launch L;
    memset(&L, 0, sizeof L);
    set_dims(&L, grid, 1, block, 1);
    L.static_shm = 4;
    L.dyn_shm = 4ull * block;
    L.nreg = 1;
    L.body = reduce_body;
    L.params = &p;
    L.buf[0] = (ox_buf){(void *)x, n, 4};
    L.buf[1] = (ox_buf){partials, grid, 4};
    L.buf[2] = (ox_buf){out, 1, 4};
    L.buf[3] = (ox_buf){&counter, 1, 4};
    L.nbuf = 4;
    L.order_seed = order_seed;
    run_opts o = {pool, bpf, {0}};
    int rc = launch(&L, &o, msg);
    if (!rc && counter != 0) {
        snprintf(msg, 192, "reduce: ticket counter not reset");
        rc = OX_ERR_CONFIG;
    }
    return rc;
}

/* ===================================================================== */
/* SCAN_I32: inclusive prefix sum mod 2^32, as three launches:            */
/*   1. per tile of B*ITEMS elements: thread-serial scan of ITEMS items,  */
/*      warp scan of thread totals with shfl_up (5 steps), warp totals    */
/*      through shared memory, scan of the warp totals by warp 0, local   */
/*      inclusive results and the tile total;                             */
/*   2. one block: exclusive scan of the tile totals (the grid carry);    */
/*   3. add each tile's carry to its elements.                            */
/* A single-pass GPU scan computes the same numbers because addition mod  */
/* 2^32 is associative and commutative.                                    */
/* ===================================================================== */
#define SC_MAXITEMS 64
/* registers: items 0..63, thread total, shuffle result, width, the value
 * being warp-scanned by the current warp region (SC_INCL for the thread
 * totals, SC_W0 for warp 0's scan of the warp totals), deltas 1..16 */
enum { SC_TOT = SC_MAXITEMS, SC_TMP, SC_WID, SC_INCL, SC_W0, SC_D0, SC_NREG = SC_D0 + 5 };

typedef struct {
    uint32_t n, items;
    uint64_t ntiles;
} scan_params;

static uint64_t sc_base(ox_block *b, uint32_t t) {
    const scan_params *p = b->params;
    return (uint64_t)b->bidx[0] * b->block[0] * p->items + (uint64_t)t * p->items;
}

static void sc_set_deltas(ox_block *b, uint32_t t) {
    ox_w32(b, t, SC_WID, 32);
    for (int s = 0; s < 5; s++) ox_w32(b, t, SC_D0 + s, 1u << s);
}

/* thread-serial inclusive scan of the thread's ITEMS consecutive items */
static int sc_thread_items(ox_block *b, uint32_t t) {
    const scan_params *p = b->params;
    uint64_t base = sc_base(b, t);
    uint32_t run = 0;
    for (uint32_t k = 0; k < p->items; k++) {
        uint64_t i = base + k;
        run += (i < p->n) ? ox_g_ld32(b, 0, i) : 0u;
        ox_w32(b, t, (int)k, run);
    }
    ox_w32(b, t, SC_TOT, run);
    ox_w32(b, t, SC_INCL, run);
    sc_set_deltas(b, t);
    return 0;
}

/* after y = shfl_up(x, D): if lane >= D, x += y (one Hillis-Steele step) */
#define SC_ACC(D)                                                                          \
    static int sc_acc##D(ox_block *b, uint32_t t) {                                        \
        if ((t & 31u) >= D) ox_w32(b, t, SC_INCL, ox_r32(b, t, SC_INCL) + ox_r32(b, t, SC_TMP)); \
        return 0;                                                                          \
    }                                                                                      \
    static int sc_w0acc##D(ox_block *b, uint32_t t) {                                      \
        if (t < 32u && (t & 31u) >= D) ox_w32(b, t, SC_W0, ox_r32(b, t, SC_W0) + ox_r32(b, t, SC_TMP)); \
        return 0;                                                                          \
    }
SC_ACC(1)
SC_ACC(2)
SC_ACC(4)
SC_ACC(8)
SC_ACC(16)

/* warp-inclusive scan of register SC_INCL: five shfl_up steps, the first
 * lane loop being `first` */
static void sc_warp_scan(ox_block *b, ox_thread_fn first, int warp0) {
    int r = warp0 ? SC_W0 : SC_INCL;
    ox_warp_step st[6] = {
        {first, OX_W_UP, r, SC_D0 + 0, SC_WID, SC_TMP},
        {warp0 ? sc_w0acc1 : sc_acc1, OX_W_UP, r, SC_D0 + 1, SC_WID, SC_TMP},
        {warp0 ? sc_w0acc2 : sc_acc2, OX_W_UP, r, SC_D0 + 2, SC_WID, SC_TMP},
        {warp0 ? sc_w0acc4 : sc_acc4, OX_W_UP, r, SC_D0 + 3, SC_WID, SC_TMP},
        {warp0 ? sc_w0acc8 : sc_acc8, OX_W_UP, r, SC_D0 + 4, SC_WID, SC_TMP},
        {warp0 ? sc_w0acc16 : sc_acc16, OX_W_NONE, 0, -1, -1, 0},
    };
    ox_warp_region(b, st, 6);
}

/* the last lane of each warp publishes the warp total */
static int sc_store_warp_total(ox_block *b, uint32_t t) {
    if ((t & 31u) == 31u) ox_s_st32(b, 4ull * (t >> 5), ox_r32(b, t, SC_INCL));
    return 0;
}

/* warp 0 loads the warp totals (zero beyond the block's warp count) */
static int sc_warp0_load(ox_block *b, uint32_t t) {
    uint32_t nw = b->block[0] / 32u;
    ox_w32(b, t, SC_W0, (t < nw) ? ox_s_ld32(b, 4ull * t) : 0u);
    sc_set_deltas(b, t);
    return 0;
}

static int sc_warp0_store(ox_block *b, uint32_t t) {
    uint32_t nw = b->block[0] / 32u;
    if (t < nw) ox_s_st32(b, 4ull * t, ox_r32(b, t, SC_W0));
    return 0;
}

static int sc_write_local(ox_block *b, uint32_t t) {
    const scan_params *p = b->params;
    uint32_t w = t >> 5;
    uint32_t prefix = (w ? ox_s_ld32(b, 4ull * (w - 1)) : 0u) + ox_r32(b, t, SC_INCL) - ox_r32(b, t, SC_TOT);
    uint64_t base = sc_base(b, t);
    for (uint32_t k = 0; k < p->items; k++) {
        uint64_t i = base + k;
        if (i < p->n) ox_g_st32(b, 1, i, prefix + ox_r32(b, t, (int)k));
    }
    if (t == 0) ox_g_st32(b, 2, b->bidx[0], ox_s_ld32(b, 4ull * (b->block[0] / 32u - 1)));
    return 0;
}

static void scan_tiles_body(ox_block *b) {
    sc_warp_scan(b, sc_thread_items, 0);    /* warp-level: no barrier      */
    ox_threads(b, sc_store_warp_total);     /* ... __syncthreads()         */
    sc_warp_scan(b, sc_warp0_load, 1);      /* warp 0 scans the totals     */
    ox_threads(b, sc_warp0_store);          /* ... __syncthreads()         */
    ox_threads(b, sc_write_local);
}

/* launch 2: one block, exclusive scan of the tile totals in chunks of B,
 * a shared-memory Hillis-Steele scan per chunk, running carry in shared
 * word B (written by thread 0). */
static int ss_load(ox_block *b, uint32_t t) {
    const scan_params *p = b->params;
    uint64_t i = (uint64_t)b->u[2] * b->block[0] + t;
    ox_s_st32(b, 4ull * t, i < p->ntiles ? ox_g_ld32(b, 2, i) : 0u);
    if (b->u[2] == 0 && t == 0) ox_s_st32(b, 4ull * 2 * b->block[0], 0u);
    return 0;
}
/* double-buffered step: read from half `u[3]`, write the other half */
static int ss_step(ox_block *b, uint32_t t) {
    uint32_t B = b->block[0];
    uint32_t d = U32(b->u[1]);
    uint64_t src = b->u[3] ? B : 0, dst = b->u[3] ? 0 : B;
    uint32_t v = ox_s_ld32(b, 4ull * (src + t));
    if (t >= d) v += ox_s_ld32(b, 4ull * (src + t - d));
    ox_s_st32(b, 4ull * (dst + t), v);
    return 0;
}
static int ss_write(ox_block *b, uint32_t t) {
    const scan_params *p = b->params;
    uint32_t B = b->block[0];
    uint64_t cur = b->u[3] ? B : 0; /* half holding the inclusive scan */
    uint64_t i = (uint64_t)b->u[2] * B + t;
    uint32_t carry = ox_s_ld32(b, 4ull * 2 * B);
    uint32_t incl = ox_s_ld32(b, 4ull * (cur + t));
    uint32_t own = i < p->ntiles ? ox_g_ld32(b, 2, i) : 0u;
    if (i < p->ntiles) ox_g_st32(b, 3, i, carry + incl - own);
    return 0;
}
static int ss_carry(ox_block *b, uint32_t t) {
    uint32_t B = b->block[0];
    uint64_t cur = b->u[3] ? B : 0;
    if (t == 0) ox_s_st32(b, 4ull * 2 * B, ox_s_ld32(b, 4ull * 2 * B) + ox_s_ld32(b, 4ull * (cur + B - 1)));
    return 0;
}

static void scan_sums_body(ox_block *b) {
    const scan_params *p = b->params;
    uint32_t B = b->block[0];
    uint64_t chunks = (p->ntiles + B - 1) / B;
    for (uint64_t c = 0; c < chunks; c++) {
        b->u[2] = (int64_t)c;
        ox_threads(b, ss_load);
        b->u[3] = 0;
        for (uint32_t d = 1; d < B; d *= 2) {
            b->u[1] = d;
            ox_threads(b, ss_step);
            b->u[3] ^= 1;
        }
        ox_threads(b, ss_write);
        ox_threads(b, ss_carry);
    }
}

static int sa_add(ox_block *b, uint32_t t) {
    const scan_params *p = b->params;
    uint32_t carry = ox_g_ld32(b, 3, b->bidx[0]);
    uint64_t base = sc_base(b, t);
    for (uint32_t k = 0; k < p->items; k++) {
        uint64_t i = base + k;
        if (i < p->n) ox_g_st32(b, 1, i, ox_g_ld32(b, 1, i) + carry);
    }
    return 0;
}
static void scan_add_body(ox_block *b) { ox_threads(b, sa_add); }

int oracle_scan_i32(const int32_t *x, uint32_t n, uint32_t block, uint32_t items, int32_t *y,
                    uint64_t order_seed, int pool, char *msg) {
    if (block == 0 || block > 1024 || (block & 31u) || items == 0 || items > SC_MAXITEMS) {
        snprintf(msg, 192, "scan: bad launch shape");
        return OX_ERR_CONFIG;
    }
    if (n == 0) return OX_OK;
    uint64_t tile = (uint64_t)block * items;
    uint64_t ntiles = (n + tile - 1) / tile;
    scan_params p = {n, items, ntiles};
    uint32_t *sums = calloc(ntiles, 4), *carry = calloc(ntiles, 4);
    if (!sums || !carry) {
        free(sums);
        free(carry);
        return OX_ERR_NOMEM;
    }
    ox_launch L;
    memset(&L, 0, sizeof L);
    L.params = &p;
    L.buf[0] = (ox_buf){(void *)x, n, 4};
    L.buf[1] = (ox_buf){y, n, 4};
    L.buf[2] = (ox_buf){sums, ntiles, 4};
    L.buf[3] = (ox_buf){carry, ntiles, 4};
    L.nbuf = 4;
    L.order_seed = order_seed;
    run_opts o = {pool, 0, {0}};
    /* launch 1 */
    set_dims(&L, U32(ntiles), 1, block, 1);
    L.static_shm = 4ull * 32;
    L.nreg = SC_NREG;
    L.body = scan_tiles_body;
    int rc = launch(&L, &o, msg);
    /* launch 2 */
    if (!rc) {
        set_dims(&L, 1, 1, block, 1);
        L.static_shm = 4ull * (2 * block + 1);
        L.nreg = 1;
        L.body = scan_sums_body;
        rc = launch(&L, &o, msg);
    }
    /* launch 3 */
    if (!rc) {
        set_dims(&L, U32(ntiles), 1, block, 1);
        L.static_shm = 0;
        L.nreg = 1;
        L.body = scan_add_body;
        rc = launch(&L, &o, msg);
    }
    free(sums);
    free(carry);
    return rc;
}

/* ===================================================================== */
/* HIST256_U32: per-block shared sub-histogram with shared atomics, then  */
/* a flush of the non-zero bins with global atomics.  The host zeroes    */
/* hist before the launch (the class overwrites hist).                    */
/*   buffers: 0 keys[n], 1 hist[256]; shared s[256]                       */
/*   Block b owns keys[b*S, min((b+1)*S, n)), S = 4*ceil(n / (4*G)).      */
/* ===================================================================== */
typedef struct {
    uint32_t n, seg;
} hist_params;

static int hs_zero(ox_block *b, uint32_t t) {
    for (uint32_t i = t; i < 256; i += b->block[0]) ox_s_st32(b, 4ull * i, 0u);
    return 0;
}
static int hs_count(ox_block *b, uint32_t t) {
    const hist_params *p = b->params;
    uint64_t lo = (uint64_t)b->bidx[0] * p->seg;
    uint64_t hi = lo + p->seg < p->n ? lo + p->seg : p->n;
    for (uint64_t j = lo + t; j < hi; j += b->block[0]) ox_sh_atomic_add32(b, 4ull * (ox_g_ld32(b, 0, j) & 255u), 1u);
    return 0;
}
static int hs_flush(ox_block *b, uint32_t t) {
    for (uint32_t i = t; i < 256; i += b->block[0]) {
        uint32_t c = ox_s_ld32(b, 4ull * i);
        if (c) ox_g_atomic_add32(b, 1, i, c);
    }
    return 0;
}
static void hist_body(ox_block *b) {
    ox_threads(b, hs_zero);
    ox_threads(b, hs_count);
    ox_threads(b, hs_flush);
}

int oracle_hist256_u32(const uint32_t *keys, uint32_t n, uint32_t grid, uint32_t block, uint32_t *hist,
                       uint64_t order_seed, int pool, uint32_t bpf, char *msg) {
    if (grid == 0 || block == 0 || block > 1024) {
        snprintf(msg, 192, "hist: bad launch shape");
        return OX_ERR_CONFIG;
    }
    memset(hist, 0, 256 * 4);
    hist_params p = {n, 4u * U32((n + 4ull * grid - 1) / (4ull * grid))};
    ox_launch L;
    memset(&L, 0, sizeof L);
    set_dims(&L, grid, 1, block, 1);
    L.static_shm = 256 * 4;
    L.nreg = 1;
    L.body = hist_body;
    L.params = &p;
    L.buf[0] = (ox_buf){(void *)keys, n, 4};
    L.buf[1] = (ox_buf){hist, 256, 4};
    L.nbuf = 2;
    L.order_seed = order_seed;
    run_opts o = {pool, bpf, {0}};
    return launch(&L, &o, msg);
}

/* ===================================================================== */
/* JACOBI5_F32: one sweep of the 5-point Laplace-Jacobi stencil.          */
/*   u'[i][j] = 0.25f * ((u[i-1][j] + u[i+1][j]) + (u[i][j-1] + u[i][j+1]))*/
/*   for interior cells, border cells copied.  Row-major, ny rows of nx.  */
/*   A BX x BY block stages its tile plus a one-cell halo in shared       */
/*   memory ((BY+2) x (BX+2) floats), barrier, then computes.             */
/*   buffers: 0 u[nx*ny], 1 u_next[nx*ny]                                 */
/* ===================================================================== */
typedef struct {
    uint32_t nx, ny;
} jac_params;

static uint64_t jt_off(ox_block *b, uint32_t r, uint32_t c) { return 4ull * ((uint64_t)r * (b->block[0] + 2) + c); }

static int jc_load(ox_block *b, uint32_t t) {
    const jac_params *p = b->params;
    uint32_t BX = b->block[0], BY = b->block[1];
    uint32_t tx = t % BX, ty = t / BX;
    uint64_t j = (uint64_t)b->bidx[0] * BX + tx, i = (uint64_t)b->bidx[1] * BY + ty;
    if (i >= p->ny || j >= p->nx) return 0;
    uint64_t nx = p->nx;
    ox_s_stf(b, jt_off(b, ty + 1, tx + 1), ox_g_ldf(b, 0, i * nx + j));
    if (tx == 0 && j > 0) ox_s_stf(b, jt_off(b, ty + 1, 0), ox_g_ldf(b, 0, i * nx + j - 1));
    if (tx == BX - 1 && j + 1 < p->nx) ox_s_stf(b, jt_off(b, ty + 1, BX + 1), ox_g_ldf(b, 0, i * nx + j + 1));
    if (ty == 0 && i > 0) ox_s_stf(b, jt_off(b, 0, tx + 1), ox_g_ldf(b, 0, (i - 1) * nx + j));
    if (ty == BY - 1 && i + 1 < p->ny) ox_s_stf(b, jt_off(b, BY + 1, tx + 1), ox_g_ldf(b, 0, (i + 1) * nx + j));
    return 0;
}

static int jc_compute(ox_block *b, uint32_t t) {
    const jac_params *p = b->params;
    uint32_t BX = b->block[0], BY = b->block[1];
    uint32_t tx = t % BX, ty = t / BX;
    uint64_t j = (uint64_t)b->bidx[0] * BX + tx, i = (uint64_t)b->bidx[1] * BY + ty;
    if (i >= p->ny || j >= p->nx) return 0;
    float c = ox_s_ldf(b, jt_off(b, ty + 1, tx + 1));
    float v;
    if (i == 0 || j == 0 || i == p->ny - 1 || j == p->nx - 1) {
        v = c;
    } else {
        float nn = ox_s_ldf(b, jt_off(b, ty, tx + 1));
        float ss = ox_s_ldf(b, jt_off(b, ty + 2, tx + 1));
        float ww = ox_s_ldf(b, jt_off(b, ty + 1, tx));
        float ee = ox_s_ldf(b, jt_off(b, ty + 1, tx + 2));
        float ns = nn + ss;
        float we = ww + ee;
        float sum = ns + we;
        v = 0.25f * sum;
    }
    ox_g_stf(b, 1, i * (uint64_t)p->nx + j, v);
    return 0;
}

static void jacobi_body(ox_block *b) {
    ox_threads(b, jc_load);
    ox_threads(b, jc_compute);
}

int oracle_jacobi5_f32(const float *u, float *u_next, uint32_t nx, uint32_t ny, uint32_t bx, uint32_t by,
                       uint64_t order_seed, int pool, char *msg) {
    if (nx == 0 || ny == 0 || bx == 0 || by == 0 || (uint64_t)bx * by > 1024) {
        snprintf(msg, 192, "jacobi: bad launch shape");
        return OX_ERR_CONFIG;
    }
    jac_params p = {nx, ny};
    ox_launch L;
    memset(&L, 0, sizeof L);
    set_dims(&L, (nx + bx - 1) / bx, (ny + by - 1) / by, bx, by);
    L.static_shm = 4ull * (bx + 2) * (by + 2);
    L.nreg = 1;
    L.body = jacobi_body;
    L.params = &p;
    L.buf[0] = (ox_buf){(void *)u, (uint64_t)nx * ny, 4};
    L.buf[1] = (ox_buf){u_next, (uint64_t)nx * ny, 4};
    L.nbuf = 2;
    L.order_seed = order_seed;
    run_opts o = {pool, 0, {0}};
    return launch(&L, &o, msg);
}

/* ===================================================================== */
/* GEMM_F32: C = A * B, row-major, 64x64 output tile per block of 256     */
/* threads (16x16, 4x4 outputs each), k-tiles of 16 staged in shared      */
/* memory As[64][16], Bs[16][64] with zero fill outside the matrices;     */
/* fp32 accumulation in ascending k.                                      */
/*   buffers: 0 A[M*K], 1 B[K*N], 2 C[M*N]                                */
/* ===================================================================== */
typedef struct {
    uint32_t M, N, K;
} gemm_params;
#define GT 64
#define GK 16
#define AS_OFF(r, c) (4ull * ((r) * GK + (c)))
#define BS_OFF(r, c) (4ull * (GT * GK + (r) * GT + (c)))

static int gm_init(ox_block *b, uint32_t t) {
    for (int k = 0; k < 16; k++) ox_wf(b, t, k, 0.0f);
    return 0;
}
static int gm_load(ox_block *b, uint32_t t) {
    const gemm_params *p = b->params;
    uint32_t k0 = U32(b->u[0]);
    for (uint32_t e = t; e < GT * GK; e += 256) {
        uint32_t r = e / GK, c = e % GK; /* A tile element (r, c) */
        uint64_t gi = (uint64_t)b->bidx[1] * GT + r, gk = k0 + c;
        ox_s_stf(b, AS_OFF(r, c), (gi < p->M && gk < p->K) ? ox_g_ldf(b, 0, gi * p->K + gk) : 0.0f);
        uint32_t br = e / GT, bc = e % GT; /* B tile element (br, bc) */
        uint64_t gk2 = k0 + br, gj = (uint64_t)b->bidx[0] * GT + bc;
        ox_s_stf(b, BS_OFF(br, bc), (gk2 < p->K && gj < p->N) ? ox_g_ldf(b, 1, gk2 * p->N + gj) : 0.0f);
    }
    return 0;
}
static int gm_fma(ox_block *b, uint32_t t) {
    uint32_t tx = t % 16, ty = t / 16;
    for (uint32_t kk = 0; kk < GK; kk++)
        for (uint32_t r = 0; r < 4; r++)
            for (uint32_t c = 0; c < 4; c++) {
                float a = ox_s_ldf(b, AS_OFF(ty * 4 + r, kk));
                float bb = ox_s_ldf(b, BS_OFF(kk, tx * 4 + c));
                float prod = a * bb;
                ox_wf(b, t, (int)(r * 4 + c), ox_rf(b, t, (int)(r * 4 + c)) + prod);
            }
    return 0;
}
static int gm_store(ox_block *b, uint32_t t) {
    const gemm_params *p = b->params;
    uint32_t tx = t % 16, ty = t / 16;
    for (uint32_t r = 0; r < 4; r++)
        for (uint32_t c = 0; c < 4; c++) {
            uint64_t i = (uint64_t)b->bidx[1] * GT + ty * 4 + r, j = (uint64_t)b->bidx[0] * GT + tx * 4 + c;
            if (i < p->M && j < p->N) ox_g_stf(b, 2, i * p->N + j, ox_rf(b, t, (int)(r * 4 + c)));
        }
    return 0;
}
static void gemm_body(ox_block *b) {
    const gemm_params *p = b->params;
    ox_threads(b, gm_init);
    for (uint32_t k0 = 0; k0 < p->K; k0 += GK) {
        b->u[0] = k0;
        ox_threads(b, gm_load);
        ox_threads(b, gm_fma);
    }
    ox_threads(b, gm_store);
}

int oracle_gemm_f32(const float *A, const float *B, float *C, uint32_t M, uint32_t N, uint32_t K,
                    uint64_t order_seed, int pool, char *msg) {
    if (M == 0 || N == 0 || K == 0) {
        snprintf(msg, 192, "gemm: empty shape");
        return OX_ERR_CONFIG;
    }
    gemm_params p = {M, N, K};
    ox_launch L;
    memset(&L, 0, sizeof L);
    set_dims(&L, (N + GT - 1) / GT, (M + GT - 1) / GT, 256, 1);
    L.static_shm = 4ull * 2 * GT * GK;
    L.nreg = 16;
    L.body = gemm_body;
    L.params = &p;
    L.buf[0] = (ox_buf){(void *)A, (uint64_t)M * K, 4};
    L.buf[1] = (ox_buf){(void *)B, (uint64_t)K * N, 4};
    L.buf[2] = (ox_buf){C, (uint64_t)M * N, 4};
    L.nbuf = 3;
    L.order_seed = order_seed;
    run_opts o = {pool, 0, {0}};
    return launch(&L, &o, msg);
}

/* ===================================================================== */
/* WARPTEST: conformance of the 32-lane warp operations.                  */
/*   buffers: 0 val[G*B] (int32), 1 pred[G*B] (uint32), 2 out[NC*G*B]    */
/*   Case numbering (out[c * G*B + gtid]):                                */
/*    c = (op*6 + wi)*32 + p, op 0 shfl / 1 up / 2 down / 3 xor,          */
/*        width 1 << wi (wi = 0..5), parameter p = 0..31: op(val, p, w);  */
/*    c = 768 + v*32 + j, v 0 ballot / 1 any / 2 all over predicate       */
/*        bit j of pred;                                                  */
/*    c = 864 + (o*2 + ws)*5 + q: the constant-parameter forms, op o      */
/*        (0 up, 1 down, 2 xor, 3 shfl), width 32 >> ws, p = 1 << q.      */
/* ===================================================================== */
#define WT_NRT 864
#define WT_NC 904
enum { WT_VAL, WT_PRED, WT_PAR, WT_WID, WT_RES, WT_NREG };

static void wt_case(uint32_t c, int *op, uint32_t *p, uint32_t *w, int *vote, uint32_t *bit) {
    static const int shop[4] = {OX_W_SHFL, OX_W_UP, OX_W_DOWN, OX_W_XOR};
    static const int vop[3] = {OX_W_BALLOT, OX_W_ANY, OX_W_ALL};
    static const int cop[4] = {OX_W_UP, OX_W_DOWN, OX_W_XOR, OX_W_SHFL};
    *vote = 0;
    *bit = 0;
    if (c < 768) {
        *op = shop[c / 192];
        *w = 1u << ((c / 32) % 6);
        *p = c % 32;
    } else if (c < WT_NRT) {
        *vote = 1;
        *op = vop[(c - 768) / 32];
        *bit = (c - 768) % 32;
        *p = 0;
        *w = 32;
    } else {
        uint32_t k = c - WT_NRT;
        *op = cop[k / 10];
        *w = 32u >> ((k / 5) % 2);
        *p = 1u << (k % 5);
    }
}

static int wt_setup(ox_block *b, uint32_t t) {
    uint64_t gtid = (uint64_t)b->bidx[0] * b->block[0] + t;
    int op, vote;
    uint32_t p, w, bit;
    wt_case(U32(b->u[0]), &op, &p, &w, &vote, &bit);
    ox_w32(b, t, WT_VAL, ox_g_ld32(b, 0, gtid));
    ox_w32(b, t, WT_PRED, (ox_g_ld32(b, 1, gtid) >> bit) & 1u);
    ox_w32(b, t, WT_PAR, p);
    ox_w32(b, t, WT_WID, w);
    return 0;
}
static int wt_write(ox_block *b, uint32_t t) {
    uint64_t total = (uint64_t)b->grid[0] * b->block[0];
    uint64_t gtid = (uint64_t)b->bidx[0] * b->block[0] + t;
    ox_g_st32(b, 2, (uint64_t)b->u[0] * total + gtid, ox_r32(b, t, WT_RES));
    return 0;
}
static void warptest_body(ox_block *b) {
    for (uint32_t c = 0; c < WT_NC; c++) {
        int op, vote;
        uint32_t p, w, bit;
        wt_case(c, &op, &p, &w, &vote, &bit);
        b->u[0] = c;
        ox_warp_step st[2] = {{wt_setup, op, vote ? WT_PRED : WT_VAL, WT_PAR, WT_WID, WT_RES},
                              {wt_write, OX_W_NONE, 0, -1, -1, 0}};
        ox_warp_region(b, st, 2);
    }
}

int oracle_warptest(const int32_t *val, const uint32_t *pred, uint32_t grid, uint32_t block, int32_t *out,
                    uint64_t order_seed, char *msg) {
    if (grid == 0 || block == 0 || block > 1024 || (block & 31u)) {
        snprintf(msg, 192, "warptest: bad launch shape");
        return OX_ERR_CONFIG;
    }
    uint64_t total = (uint64_t)grid * block;
    ox_launch L;
    memset(&L, 0, sizeof L);
    set_dims(&L, grid, 1, block, 1);
    L.nreg = WT_NREG;
    L.body = warptest_body;
    L.buf[0] = (ox_buf){(void *)val, total, 4};
    L.buf[1] = (ox_buf){(void *)pred, total, 4};
    L.buf[2] = (ox_buf){out, total * WT_NC, 4};
    L.nbuf = 3;
    L.order_seed = order_seed;
    return ox_run(&L, msg);
}

uint32_t oracle_warptest_ncases(void) { return WT_NC; }

/* ===================================================================== */
/* REVERSE_I32: the paper's dynamic-shared-memory example (Section III): */
/* one block of n threads, n*4 bytes of dynamic shared memory:            */
/*   s[t] = d[t]; barrier; d[t] = s[n - t - 1].                           */
/* ===================================================================== */
static int rv_load(ox_block *b, uint32_t t) {
    ox_s_st32(b, b->dyn_base + 4ull * t, ox_g_ld32(b, 0, t));
    return 0;
}
static int rv_store(ox_block *b, uint32_t t) {
    uint32_t n = b->block[0];
    ox_g_st32(b, 0, t, ox_s_ld32(b, b->dyn_base + 4ull * (n - t - 1)));
    return 0;
}
/* both statements in one thread loop: the form the kernel would take if the
 * barrier were dropped (planted race for the poison check) */
static int rv_fused(ox_block *b, uint32_t t) {
    rv_load(b, t);
    rv_store(b, t);
    return 0;
}
static void reverse_body(ox_block *b) {
    if (b->u[15]) {
        ox_threads(b, rv_fused);
        return;
    }
    ox_threads(b, rv_load);
    ox_threads(b, rv_store);
}
static void reverse_body_racy(ox_block *b) {
    b->u[15] = 1;
    reverse_body(b);
}

int oracle_reverse_i32(int32_t *d, uint32_t n, uint64_t order_seed, int skip_barrier, char *msg) {
    if (n == 0 || n > 1024) {
        snprintf(msg, 192, "reverse: block of %u threads", n);
        return OX_ERR_CONFIG;
    }
    ox_launch L;
    memset(&L, 0, sizeof L);
    set_dims(&L, 1, 1, n, 1);
    L.dyn_shm = 4ull * n;
    L.nreg = 1;
    L.body = skip_barrier ? reverse_body_racy : reverse_body;
    L.buf[0] = (ox_buf){d, n, 4};
    L.nbuf = 1;
    L.order_seed = order_seed;
    return ox_run(&L, msg);
}

/* ===================================================================== */
/* Runtime probe: an empty-bodied grid on the thread pool, to read the    */
/* fetch statistics of the runtime (Section IV-A).                        */
/* ===================================================================== */
static int nop_thread(ox_block *b, uint32_t t) {
    (void)b;
    (void)t;
    return 0;
}
static void nop_body(ox_block *b) { ox_threads(b, nop_thread); }

int oracle_pool_probe(uint32_t grid, int pool, uint32_t bpf, uint64_t *fetches, uint32_t *workers,
                      uint32_t *bpf_used, char *msg) {
    ox_launch L;
    memset(&L, 0, sizeof L);
    set_dims(&L, grid, 1, 32, 1);
    L.nreg = 1;
    L.body = nop_body;
    run_opts o = {pool, bpf, {0}};
    int rc = launch(&L, &o, msg);
    *fetches = o.st.fetches;
    *workers = o.st.workers_used;
    *bpf_used = o.st.bpf;
    return rc;
}

void oracle_pool_shutdown(void) { ox_pool_stop(); }
