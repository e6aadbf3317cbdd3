/* sanitize_check.c -- test infrastructure: a driver that runs every entry
 * point of the oracle on small inputs, for a build with AddressSanitizer
 * and UndefinedBehaviorSanitizer (tests/test_oracle_sanitize.py compiles it
 * with the oracle's sources and -fsanitize=address,undefined,
 * -fno-sanitize-recover=all).  Signed overflow is undefined in C, so the
 * scan's and reduction's wraparound rule (sums modulo 2^32, reinterpreted
 * as int32) is only enforceable if no int32 addition overflows: the inputs
 * below are chosen to wrap many times.  Each call also checks an invariant
 * the result must satisfy; the program prints "sanitize ok" and exits 0
 * when all hold.  It is not part of the library and links nothing of the
 * HIP path. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_reduce_i32(const int32_t *x, uint32_t n, uint32_t grid, uint32_t block, int32_t *partials,
                      int32_t *out, uint64_t order_seed, int pool, uint32_t bpf, int skip_barrier, char *msg);
int oracle_scan_i32(const int32_t *x, uint32_t n, uint32_t block, uint32_t items, int32_t *y, uint64_t order_seed,
                    int pool, char *msg);
int oracle_hist256_u32(const uint32_t *keys, uint32_t n, uint32_t grid, uint32_t block, uint32_t *hist,
                       uint64_t order_seed, int pool, uint32_t bpf, char *msg);
int oracle_jacobi5_f32(const float *u, float *u_next, uint32_t nx, uint32_t ny, uint32_t bx, uint32_t by,
                       uint64_t order_seed, int pool, char *msg);
int oracle_gemm_f32(const float *A, const float *B, float *C, uint32_t M, uint32_t N, uint32_t K,
                    uint64_t order_seed, int pool, char *msg);
int oracle_warptest(const int32_t *val, const uint32_t *pred, uint32_t grid, uint32_t block, int32_t *out,
                    uint64_t order_seed, char *msg);
uint32_t oracle_warptest_ncases(void);
int oracle_reverse_i32(int32_t *d, uint32_t n, uint64_t order_seed, int skip_barrier, char *msg);
int oracle_pool_probe(uint32_t grid, int pool, uint32_t bpf, uint64_t *fetches, uint32_t *workers,
                      uint32_t *bpf_used, char *msg);
void oracle_pool_shutdown(void);
int oracle_jacobi5_f64(const float *u0, uint32_t nx, uint32_t ny, uint32_t sweeps, double *out);
int oracle_jacobi5_f32_sweeps(const float *u0, uint32_t nx, uint32_t ny, uint32_t sweeps, float *out);
void oracle_gemm_f64(const float *A, const float *B, uint32_t M, uint32_t N, uint32_t K, double *C);
void oracle_gemm_f64_entries(const float *A, const float *B, uint32_t N, uint32_t K, const uint32_t *ii,
                             const uint32_t *jj, uint64_t count, double *out);
int oracle_compact_i32(const int32_t *x, uint64_t n, int32_t t, int32_t *y, uint64_t *count);

static uint64_t st = 0x243F6A8885A308D3ull;
static uint32_t rnd(void) { /* xorshift64*, arbitrary test inputs */
    st ^= st >> 12;
    st ^= st << 25;
    st ^= st >> 27;
    return (uint32_t)((st * 0x2545F4914F6CDD1Dull) >> 32);
}

static int fails = 0;
#define CHECK(c, what)                                                  \
    do {                                                                \
        if (!(c)) {                                                     \
            fprintf(stderr, "FAIL %s (line %d)\n", what, __LINE__);     \
            ++fails;                                                    \
        }                                                               \
    } while (0)

int main(void) {
    char msg[256];
    /* reduce and scan over values that wrap int32 many times */
    for (int pool = 0; pool <= 3; pool += 3) {
        const uint32_t n = 70001;
        int32_t *x = malloc(4 * n), *y = malloc(4 * n), *part = malloc(4 * 97), out = 0;
        uint32_t sum = 0;
        for (uint32_t i = 0; i < n; i++) {
            x[i] = (int32_t)(rnd() | 0x40000000u);
            sum += (uint32_t)x[i];
        }
        CHECK(oracle_reduce_i32(x, n, 97, 64, part, &out, 7, pool, pool ? 5 : 0, 0, msg) == 0, "reduce rc");
        CHECK((uint32_t)out == sum, "reduce total");
        CHECK(oracle_scan_i32(x, n, 128, 8, y, 3, pool, msg) == 0, "scan rc");
        uint32_t ok = (uint32_t)y[0] == (uint32_t)x[0];
        for (uint32_t i = 1; i < n; i++) ok &= (uint32_t)y[i] - (uint32_t)y[i - 1] == (uint32_t)x[i];
        CHECK(ok && (uint32_t)y[n - 1] == sum, "scan differences");
        uint64_t m = 0;
        CHECK(oracle_compact_i32(x, n, 0x50000000, y, &m) == 0, "compact rc");
        uint64_t want = 0;
        for (uint32_t i = 0; i < n; i++) want += x[i] > 0x50000000;
        CHECK(m == want, "compact count");
        free(x);
        free(y);
        free(part);
    }
    /* histogram */
    {
        const uint32_t n = 50003;
        uint32_t *k = malloc(4 * n), h[256];
        for (uint32_t i = 0; i < n; i++) k[i] = rnd();
        CHECK(oracle_hist256_u32(k, n, 7, 128, h, 5, 2, 3, msg) == 0, "hist rc");
        uint64_t s = 0;
        for (int b = 0; b < 256; b++) s += h[b];
        CHECK(s == n, "hist total");
        free(k);
    }
    /* Jacobi: one sweep by blocks, sweeps in f32 and f64; the linear field is a fixed point */
    {
        const uint32_t nx = 37, ny = 29;
        float *u = malloc(4 * nx * ny), *v = malloc(4 * nx * ny), *w = malloc(4 * nx * ny);
        double *d = malloc(8 * nx * ny);
        for (uint32_t i = 0; i < ny; i++)
            for (uint32_t j = 0; j < nx; j++) u[i * nx + j] = (float)(i + 2 * j);
        CHECK(oracle_jacobi5_f32(u, v, nx, ny, 16, 4, 9, 2, msg) == 0, "jacobi rc");
        CHECK(memcmp(u, v, 4 * nx * ny) == 0, "jacobi fixed point");
        CHECK(oracle_jacobi5_f32_sweeps(u, nx, ny, 5, w) == 0, "jacobi sweeps rc");
        CHECK(memcmp(u, w, 4 * nx * ny) == 0, "jacobi sweeps fixed point");
        CHECK(oracle_jacobi5_f64(u, nx, ny, 5, d) == 0, "jacobi f64 rc");
        CHECK(d[5 * nx + 7] == (double)u[5 * nx + 7], "jacobi f64 fixed point");
        free(u);
        free(v);
        free(w);
        free(d);
    }
    /* GEMM against B = I, in fp32 blocks and fp64 */
    {
        const uint32_t M = 33, N = 31, K = 31;
        float *A = malloc(4 * M * K), *B = calloc(K * N, 4), *C = malloc(4 * M * N);
        double *D = malloc(8 * M * N), e[3];
        uint32_t ii[3] = {0, 7, 32}, jj[3] = {0, 30, 5};
        for (uint32_t i = 0; i < M * K; i++) A[i] = (float)((int)(rnd() % 9) - 4);
        for (uint32_t i = 0; i < K; i++) B[i * N + i] = 1.0f;
        CHECK(oracle_gemm_f32(A, B, C, M, N, K, 1, 2, msg) == 0, "gemm rc");
        CHECK(memcmp(A, C, 4 * M * N) == 0, "gemm identity");
        oracle_gemm_f64(A, B, M, N, K, D);
        oracle_gemm_f64_entries(A, B, N, K, ii, jj, 3, e);
        for (int q = 0; q < 3; q++) CHECK(e[q] == D[ii[q] * N + jj[q]] && e[q] == A[ii[q] * K + jj[q]], "gemm f64");
        free(A);
        free(B);
        free(C);
        free(D);
    }
    /* warp conformance and the dynamic-shared-memory example */
    {
        const uint32_t grid = 2, block = 64, T = grid * block, nc = oracle_warptest_ncases();
        int32_t *val = malloc(4 * T), *out = malloc(4ull * nc * T);
        uint32_t *pred = malloc(4 * T);
        for (uint32_t t = 0; t < T; t++) {
            val[t] = (int32_t)t;
            pred[t] = rnd();
        }
        CHECK(oracle_warptest(val, pred, grid, block, out, 4, msg) == 0, "warptest rc");
        int32_t d[100];
        for (int i = 0; i < 100; i++) d[i] = i;
        CHECK(oracle_reverse_i32(d, 100, 11, 0, msg) == 0 && d[0] == 99 && d[99] == 0, "reverse");
        free(val);
        free(out);
        free(pred);
    }
    /* the runtime's fetch arithmetic: grid 16, bpf 4 -> 4 fetches */
    {
        uint64_t f = 0;
        uint32_t w = 0, b = 0;
        CHECK(oracle_pool_probe(16, 4, 4, &f, &w, &b, msg) == 0 && f == 4, "pool probe");
    }
    oracle_pool_shutdown();
    if (fails) return 1;
    printf("sanitize ok\n");
    return 0;
}
