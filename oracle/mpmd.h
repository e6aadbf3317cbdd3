/* Oracle executor: runs SPMD kernel grids on the CPU the way the paper's
 * MPMD transformation does.  TEST INFRASTRUCTURE ONLY: nothing on the
 * product path includes, links or calls this code.
 *
 * Semantics followed (paper, Section III-B and Section IV):
 *  - memory mapping (III-B1): global memory is caller-owned host arrays,
 *    reached through bounds-checked accessors; shared memory is one byte
 *    array per block; private memory is per-thread "replicated" register
 *    slots that live across phases;
 *  - extra variables (III-B2): blockIdx / blockDim / gridDim and the
 *    dynamic shared-memory base are runtime-set fields of the block context;
 *  - SPMD-to-MPMD (III-B3): a block body is a sequence of thread loops, one
 *    per barrier-delimited region (loop fission at __syncthreads); code with
 *    warp-level operations runs as nested loops, an outer loop over the
 *    ceil(blockDim/32) warps and inner 32-lane loops split at each warp op;
 *  - runtime (IV): a thread pool created once, a FIFO task queue guarded by
 *    a mutex and a condition variable, fetching `bpf` blocks per atomic
 *    fetch, average coarse-grained fetching bpf = ceil(grid / pool) (IV-A1).
 *
 * Checks that turn races and undefined behaviour into errors:
 *  - every thread loop visits threads in a seeded random order; warps and
 *    lanes likewise; blocks likewise when run serially;
 *  - shared memory starts as poison and a per-byte written map makes a read
 *    before any write an error (dynamic shared memory comes from malloc in
 *    the paper, so its contents are undefined);
 *  - every global and shared access is bounds-checked;
 *  - every thread of a region must return the same control token at the
 *    region's closing barrier, and every lane of a warp op the same width.
 */
#ifndef SPMD_ORACLE_MPMD_H
#define SPMD_ORACLE_MPMD_H

#include <stddef.h>
#include <stdint.h>

#define OX_MAX_BUFS 8
#define OX_MAX_UNIFORM 16
#define OX_WARP 32

enum {
    OX_OK = 0,
    OX_ERR_BOUNDS = -1,      /* global or shared access out of bounds      */
    OX_ERR_UNINIT = -2,      /* shared-memory read before any write         */
    OX_ERR_DIVERGENT = -3,   /* threads disagree at a barrier or warp op    */
    OX_ERR_CONFIG = -4,      /* launch shape the program cannot run         */
    OX_ERR_NOMEM = -5,
};

/* One bound global buffer: host pointer, element count, element size. */
typedef struct {
    void *p;
    uint64_t n;
    uint32_t esize;
} ox_buf;

typedef struct ox_block ox_block;
/* A thread-loop body: runs one thread's share of one region and returns a
 * control token that must be equal for all threads of the region. */
typedef int (*ox_thread_fn)(ox_block *b, uint32_t tid);
typedef void (*ox_block_fn)(ox_block *b);

/* Warp operations evaluated between lane loops. */
enum {
    OX_W_NONE = 0,
    OX_W_SHFL,     /* v[seg + (p mod w)]                                   */
    OX_W_UP,       /* i < p ? own : v[lane - p]                             */
    OX_W_DOWN,     /* i + p >= w ? own : v[lane + p]                        */
    OX_W_XOR,      /* j = lane ^ p; j <= seg + w - 1 ? v[j] : own (j may be  */
                   /* in an earlier segment, as CUDA documents)              */
    OX_W_BALLOT,   /* sum over lanes of (pred != 0) << lane                 */
    OX_W_ANY,      /* ballot != 0                                           */
    OX_W_ALL,      /* ballot == 0xFFFFFFFF                                  */
};

/* One step of a warp region: run `seg` for the 32 lanes of a warp, then
 * evaluate warp op `op` reading each lane's register `src` (value or
 * predicate) and `par` (per-lane parameter), uniform width from register
 * `wid`, writing register `dst`. */
typedef struct {
    ox_thread_fn seg;
    int op;
    int src, par, wid, dst;
} ox_warp_step;

struct ox_block {
    /* launch shape and the block being executed (runtime-set variables) */
    uint32_t grid[3], block[3];
    uint32_t bidx[3];
    uint32_t nthreads;
    uint64_t linear_bid;
    /* shared memory: static + dynamic, poisoned, with a written map */
    uint8_t *shm;
    uint8_t *shm_w;
    size_t shm_bytes;
    size_t dyn_base; /* offset of the dynamic part */
    /* global memory bindings */
    ox_buf buf[OX_MAX_BUFS];
    int nbuf;
    /* replicated private registers: reg[tid * nreg + k] */
    uint64_t *reg;
    int nreg;
    /* block-uniform values set by the block driver (loop counters etc.) */
    int64_t u[OX_MAX_UNIFORM];
    /* class parameters (read-only, shared by all blocks of a launch) */
    const void *params;
    /* ordering */
    uint64_t order_seed;
    uint64_t region_counter;
    uint32_t *perm;
    /* status */
    int err;
    char msg[192];
};

/* ---- accessors used by thread bodies ---------------------------------- */
uint32_t ox_g_ld32(ox_block *b, int buf, uint64_t i);
void ox_g_st32(ox_block *b, int buf, uint64_t i, uint32_t v);
uint32_t ox_g_atomic_add32(ox_block *b, int buf, uint64_t i, uint32_t v);
float ox_g_ldf(ox_block *b, int buf, uint64_t i);
void ox_g_stf(ox_block *b, int buf, uint64_t i, float v);

uint32_t ox_s_ld32(ox_block *b, uint64_t byte_off);
void ox_s_st32(ox_block *b, uint64_t byte_off, uint32_t v);
uint32_t ox_sh_atomic_add32(ox_block *b, uint64_t byte_off, uint32_t v);
float ox_s_ldf(ox_block *b, uint64_t byte_off);
void ox_s_stf(ox_block *b, uint64_t byte_off, float v);

static inline uint64_t *ox_reg(ox_block *b, uint32_t tid, int k) {
    return &b->reg[(uint64_t)tid * (uint64_t)b->nreg + (uint64_t)k];
}
static inline uint32_t ox_r32(ox_block *b, uint32_t tid, int k) {
    return (uint32_t)*ox_reg(b, tid, k);
}
static inline void ox_w32(ox_block *b, uint32_t tid, int k, uint32_t v) {
    *ox_reg(b, tid, k) = v;
}
float ox_rf(ox_block *b, uint32_t tid, int k);
void ox_wf(ox_block *b, uint32_t tid, int k, float v);

void ox_fail(ox_block *b, int code, const char *msg);

/* ---- region drivers used by block bodies ------------------------------ */
/* One barrier-delimited region: the thread loop of the MPMD form. */
void ox_threads(ox_block *b, ox_thread_fn fn);
/* A warp region: for each warp (outer loop), run the steps' lane loops and
 * warp ops in sequence (inner loops), as in the paper's nested loops. */
void ox_warp_region(ox_block *b, const ox_warp_step *steps, int nsteps);

/* ---- launching a grid ------------------------------------------------- */
typedef struct {
    uint32_t grid[3], block[3];
    size_t static_shm, dyn_shm;
    int nreg;
    ox_block_fn body;
    const void *params;
    ox_buf buf[OX_MAX_BUFS];
    int nbuf;
    uint64_t order_seed; /* 0: natural order everywhere */
} ox_launch;

/* Runtime statistics of the thread-pool executor (Section IV). */
typedef struct {
    uint64_t fetches;        /* atomic fetches from the task queue          */
    uint32_t workers_used;   /* pool threads that executed at least 1 block */
    uint32_t bpf;            /* blocks per fetch actually used              */
} ox_stats;

/* Serial executor: blocks in linear order (x fastest) or a seeded
 * permutation.  Returns OX_OK or an error code; `msg` (>= 192 bytes) gets
 * a description. */
int ox_run(const ox_launch *L, char *msg);

/* Thread-pool executor following the paper's runtime: pool of `pool`
 * workers created once, mutex-guarded FIFO queue, `bpf` blocks per fetch
 * (0 means average coarse-grained fetching, ceil(grid / pool)). */
int ox_pool_start(int pool);
void ox_pool_stop(void);
int ox_pool_run(const ox_launch *L, uint32_t bpf, ox_stats *st, char *msg);

/* Fetch arithmetic of the runtime (Section IV-A): number of fetches and
 * of workers that receive work for a grid of `total` blocks. */
uint64_t ox_fetch_count(uint64_t total, uint64_t bpf);
uint32_t ox_average_bpf(uint64_t total, uint32_t pool);

#endif
