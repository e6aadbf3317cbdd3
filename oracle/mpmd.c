/* Oracle executor (TEST INFRASTRUCTURE ONLY): MPMD execution of SPMD
 * kernel grids on the CPU.  See mpmd.h for the semantics and the paper
 * passages each part follows. */
#include "mpmd.h"

#include <pthread.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define POISON 0xA5u

/* --------------------------------------------------------------------- */
/* order randomisation: the oracle's own SplitMix64, used only to pick    */
/* visiting orders (never to make inputs)                                  */
/* --------------------------------------------------------------------- */
static uint64_t ox_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static void ox_perm(uint32_t *p, uint32_t n, uint64_t seed, uint64_t a, uint64_t c) {
    for (uint32_t i = 0; i < n; i++) p[i] = i;
    if (seed == 0 || n < 2) return;
    uint64_t s = ox_mix(seed ^ ox_mix(a * 0x9E3779B97F4A7C15ull + c));
    for (uint32_t i = n - 1; i > 0; i--) {
        s += 0x9E3779B97F4A7C15ull;
        uint32_t j = (uint32_t)(ox_mix(s) % (uint64_t)(i + 1));
        uint32_t t = p[i];
        p[i] = p[j];
        p[j] = t;
    }
}

void ox_fail(ox_block *b, int code, const char *msg) {
    if (b->err) return;
    b->err = code;
    snprintf(b->msg, sizeof b->msg, "block (%u,%u,%u): %s", b->bidx[0], b->bidx[1], b->bidx[2], msg);
}

/* --------------------------------------------------------------------- */
/* global memory (heap in the paper's mapping)                             */
/* --------------------------------------------------------------------- */
static void *gaddr(ox_block *b, int buf, uint64_t i, uint32_t esize) {
    if (b->err) return NULL;
    if (buf < 0 || buf >= b->nbuf || b->buf[buf].esize != esize || i >= b->buf[buf].n) {
        char m[96];
        snprintf(m, sizeof m, "global access out of bounds: buffer %d index %llu", buf,
                 (unsigned long long)i);
        ox_fail(b, OX_ERR_BOUNDS, m);
        return NULL;
    }
    return (uint8_t *)b->buf[buf].p + i * esize;
}

uint32_t ox_g_ld32(ox_block *b, int buf, uint64_t i) {
    uint32_t *p = gaddr(b, buf, i, 4);
    return p ? *p : 0u;
}
void ox_g_st32(ox_block *b, int buf, uint64_t i, uint32_t v) {
    uint32_t *p = gaddr(b, buf, i, 4);
    if (p) *p = v;
}
uint32_t ox_g_atomic_add32(ox_block *b, int buf, uint64_t i, uint32_t v) {
    uint32_t *p = gaddr(b, buf, i, 4);
    return p ? __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST) : 0u;
}
float ox_g_ldf(ox_block *b, int buf, uint64_t i) {
    float *p = gaddr(b, buf, i, 4);
    return p ? *p : 0.0f;
}
void ox_g_stf(ox_block *b, int buf, uint64_t i, float v) {
    float *p = gaddr(b, buf, i, 4);
    if (p) *p = v;
}

/* --------------------------------------------------------------------- */
/* shared memory (one array per block, poisoned, written-map checked)     */
/* --------------------------------------------------------------------- */
static uint8_t *saddr(ox_block *b, uint64_t off, int reading) {
    if (b->err) return NULL;
    if (off + 4 > b->shm_bytes || (off & 3)) {
        char m[96];
        snprintf(m, sizeof m, "shared access out of bounds: byte %llu of %zu",
                 (unsigned long long)off, b->shm_bytes);
        ox_fail(b, OX_ERR_BOUNDS, m);
        return NULL;
    }
    if (reading) {
        for (int k = 0; k < 4; k++)
            if (!b->shm_w[off + k]) {
                char m[96];
                snprintf(m, sizeof m, "shared read before write at byte %llu", (unsigned long long)off);
                ox_fail(b, OX_ERR_UNINIT, m);
                return NULL;
            }
    }
    return b->shm + off;
}

uint32_t ox_s_ld32(ox_block *b, uint64_t off) {
    uint8_t *p = saddr(b, off, 1);
    uint32_t v = 0;
    if (p) memcpy(&v, p, 4);
    return v;
}
void ox_s_st32(ox_block *b, uint64_t off, uint32_t v) {
    uint8_t *p = saddr(b, off, 0);
    if (!p) return;
    memcpy(p, &v, 4);
    memset(b->shm_w + off, 1, 4);
}
uint32_t ox_sh_atomic_add32(ox_block *b, uint64_t off, uint32_t v) {
    /* threads of one block run one at a time, so a read-modify-write is
     * already atomic with respect to the block */
    uint32_t old = ox_s_ld32(b, off);
    ox_s_st32(b, off, old + v);
    return old;
}
float ox_s_ldf(ox_block *b, uint64_t off) {
    uint32_t u = ox_s_ld32(b, off);
    float f;
    memcpy(&f, &u, 4);
    return f;
}
void ox_s_stf(ox_block *b, uint64_t off, float v) {
    uint32_t u;
    memcpy(&u, &v, 4);
    ox_s_st32(b, off, u);
}

float ox_rf(ox_block *b, uint32_t tid, int k) {
    uint32_t u = ox_r32(b, tid, k);
    float f;
    memcpy(&f, &u, 4);
    return f;
}
void ox_wf(ox_block *b, uint32_t tid, int k, float v) {
    uint32_t u;
    memcpy(&u, &v, 4);
    ox_w32(b, tid, k, u);
}

/* --------------------------------------------------------------------- */
/* regions                                                                 */
/* --------------------------------------------------------------------- */
void ox_threads(ox_block *b, ox_thread_fn fn) {
    if (b->err) return;
    uint32_t n = b->nthreads;
    ox_perm(b->perm, n, b->order_seed, b->linear_bid, b->region_counter++);
    int tok0 = 0;
    for (uint32_t k = 0; k < n; k++) {
        int tok = fn(b, b->perm[k]);
        if (b->err) return;
        if (k == 0)
            tok0 = tok;
        else if (tok != tok0) {
            ox_fail(b, OX_ERR_DIVERGENT, "threads reach the closing barrier on different paths");
            return;
        }
    }
}

/* CUDA warp-op semantics on one 32-lane warp (CUDA programming guide and
 * the PTX ISA description of shfl.sync: source lane, clamp to the lane's
 * width-segment, out-of-segment reads return the caller's own value). */
static uint32_t warp_eval(int op, const uint32_t *v, uint32_t lane, uint32_t p, uint32_t w,
                          uint32_t ballot) {
    uint32_t seg = lane & ~(w - 1);
    uint32_t i = lane & (w - 1);
    uint32_t last = seg + w - 1;
    p &= 31u; /* the lane offset / mask / source operand is taken mod 32 */
    switch (op) {
    case OX_W_SHFL:
        return v[seg + (p & (w - 1))];
    case OX_W_UP:
        return (i < p) ? v[lane] : v[lane - p];
    case OX_W_DOWN:
        return (i + p >= w) ? v[lane] : v[lane + p];
    case OX_W_XOR: {
        uint32_t j = lane ^ p; /* may land in an earlier segment: allowed */
        return (j <= last) ? v[j] : v[lane];
    }
    case OX_W_BALLOT:
        return ballot;
    case OX_W_ANY:
        return ballot != 0u;
    case OX_W_ALL:
        return ballot == 0xFFFFFFFFu;
    }
    return 0;
}

void ox_warp_region(ox_block *b, const ox_warp_step *steps, int nsteps) {
    if (b->err) return;
    uint32_t n = b->nthreads;
    uint32_t nw = (n + OX_WARP - 1) / OX_WARP;
    uint32_t *wperm = malloc(sizeof(uint32_t) * nw);
    if (!wperm) {
        ox_fail(b, OX_ERR_NOMEM, "out of memory");
        return;
    }
    ox_perm(wperm, nw, b->order_seed, b->linear_bid, b->region_counter++);
    uint32_t lperm[OX_WARP];
    for (uint32_t wi = 0; wi < nw && !b->err; wi++) {
        uint32_t w = wperm[wi];
        uint32_t base = w * OX_WARP;
        uint32_t lanes = (n - base < OX_WARP) ? n - base : OX_WARP;
        for (int s = 0; s < nsteps && !b->err; s++) {
            const ox_warp_step *st = &steps[s];
            if (st->seg) {
                ox_perm(lperm, lanes, b->order_seed, b->linear_bid * 65537u + w, b->region_counter++);
                int tok0 = 0;
                for (uint32_t k = 0; k < lanes; k++) {
                    int tok = st->seg(b, base + lperm[k]);
                    if (b->err) break;
                    if (k == 0)
                        tok0 = tok;
                    else if (tok != tok0)
                        ox_fail(b, OX_ERR_DIVERGENT, "lanes reach a warp op on different paths");
                }
            }
            if (b->err || st->op == OX_W_NONE) continue;
            if (lanes != OX_WARP) {
                ox_fail(b, OX_ERR_CONFIG, "warp op in a partial warp");
                break;
            }
            uint32_t v[OX_WARP], par[OX_WARP], width = 32, ballot = 0;
            for (uint32_t l = 0; l < OX_WARP; l++) {
                v[l] = ox_r32(b, base + l, st->src);
                par[l] = st->par >= 0 ? ox_r32(b, base + l, st->par) : 0u;
                uint32_t wl = st->wid >= 0 ? ox_r32(b, base + l, st->wid) : 32u;
                if (l == 0)
                    width = wl;
                else if (wl != width)
                    ox_fail(b, OX_ERR_DIVERGENT, "lanes disagree on the shuffle width");
                if (v[l] != 0u) ballot |= 1u << l;
            }
            if (width == 0 || width > 32 || (width & (width - 1))) {
                ox_fail(b, OX_ERR_CONFIG, "shuffle width is not a power of two in [1,32]");
                break;
            }
            uint32_t res[OX_WARP];
            for (uint32_t l = 0; l < OX_WARP; l++) res[l] = warp_eval(st->op, v, l, par[l], width, ballot);
            for (uint32_t l = 0; l < OX_WARP; l++) ox_w32(b, base + l, st->dst, res[l]);
        }
    }
    free(wperm);
}

/* --------------------------------------------------------------------- */
/* block contexts                                                          */
/* --------------------------------------------------------------------- */
typedef struct {
    ox_block b;
    size_t shm_cap;
    uint64_t reg_cap;
    uint32_t perm_cap;
} ox_ctx;

static int ctx_prepare(ox_ctx *c, const ox_launch *L) {
    uint32_t nt = L->block[0] * L->block[1] * L->block[2];
    size_t shm = L->static_shm + L->dyn_shm;
    uint64_t regs = (uint64_t)nt * (uint64_t)(L->nreg > 0 ? L->nreg : 1);
    if (shm > c->shm_cap) {
        free(c->b.shm);
        free(c->b.shm_w);
        c->b.shm = malloc(shm ? shm : 1);
        c->b.shm_w = malloc(shm ? shm : 1);
        c->shm_cap = shm;
        if (!c->b.shm || !c->b.shm_w) return OX_ERR_NOMEM;
    }
    if (regs > c->reg_cap) {
        free(c->b.reg);
        c->b.reg = malloc(regs * sizeof(uint64_t));
        c->reg_cap = regs;
        if (!c->b.reg) return OX_ERR_NOMEM;
    }
    if (nt > c->perm_cap) {
        free(c->b.perm);
        c->b.perm = malloc(nt * sizeof(uint32_t));
        c->perm_cap = nt;
        if (!c->b.perm) return OX_ERR_NOMEM;
    }
    memcpy(c->b.grid, L->grid, sizeof L->grid);
    memcpy(c->b.block, L->block, sizeof L->block);
    c->b.nthreads = nt;
    c->b.shm_bytes = shm;
    c->b.dyn_base = L->static_shm;
    memcpy(c->b.buf, L->buf, sizeof L->buf);
    c->b.nbuf = L->nbuf;
    c->b.nreg = L->nreg > 0 ? L->nreg : 1;
    c->b.params = L->params;
    c->b.order_seed = L->order_seed;
    c->b.err = 0;
    c->b.msg[0] = 0;
    return OX_OK;
}

static void ctx_free(ox_ctx *c) {
    free(c->b.shm);
    free(c->b.shm_w);
    free(c->b.reg);
    free(c->b.perm);
    memset(c, 0, sizeof *c);
}

/* Set the runtime variables of one block and run its body: the analogue of
 * the paper's per-block setup before calling the transformed kernel. */
static int run_block(ox_ctx *c, const ox_launch *L, uint64_t lin) {
    ox_block *b = &c->b;
    uint64_t gx = L->grid[0], gy = L->grid[1];
    b->bidx[0] = (uint32_t)(lin % gx);
    b->bidx[1] = (uint32_t)((lin / gx) % gy);
    b->bidx[2] = (uint32_t)(lin / (gx * gy));
    b->linear_bid = lin;
    b->region_counter = 0;
    memset(b->u, 0, sizeof b->u);
    /* fresh, undefined shared memory and registers (a launch without shared
     * memory has no buffer: memset of a null pointer is undefined even for
     * zero bytes) */
    if (b->shm_bytes) {
        memset(b->shm, POISON, b->shm_bytes);
        memset(b->shm_w, 0, b->shm_bytes);
    }
    memset(b->reg, 0xCD, (uint64_t)b->nthreads * b->nreg * sizeof(uint64_t));
    L->body(b);
    return b->err;
}

static int check_launch(const ox_launch *L, char *msg) {
    for (int d = 0; d < 3; d++)
        if (L->grid[d] == 0 || L->block[d] == 0) {
            snprintf(msg, 192, "zero launch dimension");
            return OX_ERR_CONFIG;
        }
    return OX_OK;
}

int ox_run(const ox_launch *L, char *msg) {
    int rc = check_launch(L, msg);
    if (rc) return rc;
    ox_ctx c;
    memset(&c, 0, sizeof c);
    rc = ctx_prepare(&c, L);
    if (rc) {
        snprintf(msg, 192, "out of memory");
        ctx_free(&c);
        return rc;
    }
    uint64_t total = (uint64_t)L->grid[0] * L->grid[1] * L->grid[2];
    uint32_t *order = NULL;
    if (L->order_seed && total <= 0xFFFFFFFFull) {
        order = malloc(total * sizeof(uint32_t));
        if (order) ox_perm(order, (uint32_t)total, L->order_seed, 0xB10Cull, 0);
    }
    for (uint64_t k = 0; k < total; k++) {
        rc = run_block(&c, L, order ? order[k] : k);
        if (rc) {
            snprintf(msg, 192, "%s", c.b.msg);
            break;
        }
    }
    free(order);
    ctx_free(&c);
    return rc;
}

/* --------------------------------------------------------------------- */
/* thread-pool runtime (Section IV): pool created once, FIFO task queue    */
/* under a mutex, condition variable to wake the pool, coarse fetching     */
/* --------------------------------------------------------------------- */
uint64_t ox_fetch_count(uint64_t total, uint64_t bpf) {
    return bpf ? (total + bpf - 1) / bpf : 0;
}

uint32_t ox_average_bpf(uint64_t total, uint32_t pool) {
    if (pool == 0) return 0;
    uint64_t b = (total + pool - 1) / pool;
    return (uint32_t)(b ? b : 1);
}

/* The task: the paper's kernel structure with the fetch cursor. */
typedef struct ox_task {
    const ox_launch *L;
    uint64_t total_blocks;
    uint64_t curr_block; /* next block to hand out */
    uint32_t bpf;
    uint64_t fetches;
    uint64_t done_blocks;
    int err;
    char msg[192];
    struct ox_task *next;
} ox_task;

static struct {
    pthread_mutex_t mu;
    pthread_cond_t wake_pool; /* workers wait here for tasks          */
    pthread_cond_t idle;      /* the host waits here for completion    */
    ox_task *head, *tail;
    pthread_t *th;
    int n;
    int stop;
    uint32_t *used; /* per worker: executed at least one block of the current task */
} P = {PTHREAD_MUTEX_INITIALIZER, PTHREAD_COND_INITIALIZER, PTHREAD_COND_INITIALIZER};

static void *worker(void *arg) {
    int id = (int)(intptr_t)arg;
    ox_ctx c;
    memset(&c, 0, sizeof c);
    for (;;) {
        pthread_mutex_lock(&P.mu);
        while (!P.stop && (P.head == NULL || P.head->curr_block >= P.head->total_blocks))
            pthread_cond_wait(&P.wake_pool, &P.mu);
        if (P.stop) {
            pthread_mutex_unlock(&P.mu);
            break;
        }
        /* fetch: advance the cursor by bpf; pop when exhausted */
        ox_task *t = P.head;
        uint64_t start = t->curr_block;
        uint64_t end = start + t->bpf;
        if (end > t->total_blocks) end = t->total_blocks; /* clamped last chunk */
        t->curr_block = end;
        t->fetches++;
        if (t->curr_block >= t->total_blocks) {
            P.head = t->next;
            if (!P.head) P.tail = NULL;
        }
        P.used[id] = 1;
        pthread_mutex_unlock(&P.mu);

        /* execute outside the lock */
        int rc = ctx_prepare(&c, t->L);
        char msg[192] = "";
        for (uint64_t k = start; k < end && rc == OX_OK; k++) {
            rc = run_block(&c, t->L, k);
            if (rc) snprintf(msg, sizeof msg, "%s", c.b.msg);
        }
        pthread_mutex_lock(&P.mu);
        t->done_blocks += end - start;
        if (rc && !t->err) {
            t->err = rc;
            snprintf(t->msg, sizeof t->msg, "%s", msg);
        }
        if (t->done_blocks == t->total_blocks) pthread_cond_broadcast(&P.idle);
        pthread_mutex_unlock(&P.mu);
    }
    ctx_free(&c);
    return NULL;
}

int ox_pool_start(int pool) {
    if (pool < 1) return OX_ERR_CONFIG;
    if (P.n == pool) return OX_OK;
    if (P.n) ox_pool_stop();
    P.th = calloc((size_t)pool, sizeof(pthread_t));
    P.used = calloc((size_t)pool, sizeof(uint32_t));
    if (!P.th || !P.used) return OX_ERR_NOMEM;
    P.stop = 0;
    P.n = pool;
    for (int i = 0; i < pool; i++) pthread_create(&P.th[i], NULL, worker, (void *)(intptr_t)i);
    return OX_OK;
}

void ox_pool_stop(void) {
    if (!P.n) return;
    pthread_mutex_lock(&P.mu);
    P.stop = 1;
    pthread_cond_broadcast(&P.wake_pool);
    pthread_mutex_unlock(&P.mu);
    for (int i = 0; i < P.n; i++) pthread_join(P.th[i], NULL);
    free(P.th);
    free(P.used);
    P.th = NULL;
    P.used = NULL;
    P.n = 0;
}

int ox_pool_run(const ox_launch *L, uint32_t bpf, ox_stats *st, char *msg) {
    int rc = check_launch(L, msg);
    if (rc) return rc;
    if (!P.n) {
        snprintf(msg, 192, "thread pool not started");
        return OX_ERR_CONFIG;
    }
    ox_task t;
    memset(&t, 0, sizeof t);
    t.L = L;
    t.total_blocks = (uint64_t)L->grid[0] * L->grid[1] * L->grid[2];
    t.bpf = bpf ? bpf : ox_average_bpf(t.total_blocks, (uint32_t)P.n);
    /* push, then broadcast wake_pool; the host does not block here */
    pthread_mutex_lock(&P.mu);
    memset(P.used, 0, sizeof(uint32_t) * (size_t)P.n);
    if (P.tail)
        P.tail->next = &t;
    else
        P.head = &t;
    P.tail = &t;
    pthread_cond_broadcast(&P.wake_pool);
    /* synchronise: wait until every block of the task has executed */
    while (t.done_blocks < t.total_blocks) pthread_cond_wait(&P.idle, &P.mu);
    uint32_t used = 0;
    for (int i = 0; i < P.n; i++) used += P.used[i];
    pthread_mutex_unlock(&P.mu);
    if (st) {
        st->fetches = t.fetches;
        st->workers_used = used;
        st->bpf = t.bpf;
    }
    if (t.err) snprintf(msg, 192, "%s", t.msg);
    return t.err;
}
