/* FP64 reference computations (TEST INFRASTRUCTURE ONLY: nothing on the
 * product path includes, links or calls this code).
 *
 * These are the plain definitions of the two floating-point kernel classes,
 * evaluated in double precision from the same fp32 inputs, and used as the
 * accuracy reference the fp32 results are measured against.
 *
 *  - Jacobi: the 5-point Laplace-Jacobi sweep, interior cells replaced by a
 *    quarter of the sum of their four neighbours, border cells held at
 *    their initial values, a fixed number of sweeps (no residual test).
 *  - GEMM: C[i][j] = sum over k ascending of (double)A[i][k] * (double)B[k][j].
 *    Products of two fp32 values are exact in double; only the summation
 *    rounds, at about 1e-13 relative for K = 4096.
 *
 * Rows are split over OpenMP threads; each output is still computed by one
 * thread in the order the definition states.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

int oracle_jacobi5_f64(const float *u0, uint32_t nx, uint32_t ny, uint32_t sweeps, double *out) {
    uint64_t cells = (uint64_t)nx * ny;
    double *a = out;
    double *b = malloc(cells * sizeof(double));
    if (!b) return -5;
    for (uint64_t k = 0; k < cells; k++) a[k] = (double)u0[k];
    memcpy(b, a, cells * sizeof(double));
    for (uint32_t s = 0; s < sweeps; s++) {
        const double *src = (s & 1u) ? b : a;
        double *dst = (s & 1u) ? a : b;
#pragma omp parallel for schedule(static)
        for (int64_t i = 1; i < (int64_t)ny - 1; i++) {
            const double *r = src + (uint64_t)i * nx;
            double *w = dst + (uint64_t)i * nx;
            for (uint64_t j = 1; j + 1 < nx; j++)
                w[j] = 0.25 * ((r[j - nx] + r[j + nx]) + (r[j - 1] + r[j + 1]));
        }
    }
    if (sweeps & 1u) memcpy(a, b, cells * sizeof(double));
    free(b);
    return 0;
}

/* fp32 Jacobi with the association the kernel class states:
 * 0.25f * ((north + south) + (west + east)), each operation rounded to fp32.
 * A whole-grid loop rather than the block executor, so that many sweeps of
 * large grids finish quickly.  Built with -ffp-contract=off, so no step is
 * fused. */
int oracle_jacobi5_f32_sweeps(const float *u0, uint32_t nx, uint32_t ny, uint32_t sweeps, float *out) {
    uint64_t cells = (uint64_t)nx * ny;
    float *a = out;
    float *b = malloc(cells * sizeof(float));
    if (!b) return -5;
    memcpy(a, u0, cells * sizeof(float));
    memcpy(b, u0, cells * sizeof(float));
    for (uint32_t s = 0; s < sweeps; s++) {
        const float *src = (s & 1u) ? b : a;
        float *dst = (s & 1u) ? a : b;
#pragma omp parallel for schedule(static)
        for (int64_t i = 1; i < (int64_t)ny - 1; i++) {
            const float *r = src + (uint64_t)i * nx;
            float *w = dst + (uint64_t)i * nx;
            for (uint64_t j = 1; j + 1 < nx; j++) {
                float ns = r[j - nx] + r[j + nx];
                float we = r[j - 1] + r[j + 1];
                float sum = ns + we;
                w[j] = 0.25f * sum;
            }
        }
    }
    if (sweeps & 1u) memcpy(a, b, cells * sizeof(float));
    free(b);
    return 0;
}

/* Whole GEMM in double, k ascending for every output. */
void oracle_gemm_f64(const float *A, const float *B, uint32_t M, uint32_t N, uint32_t K, double *C) {
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < (int64_t)M; i++) {
        double *c = C + (uint64_t)i * N;
        for (uint32_t j = 0; j < N; j++) c[j] = 0.0;
        for (uint32_t k = 0; k < K; k++) {
            double a = (double)A[(uint64_t)i * K + k];
            const float *brow = B + (uint64_t)k * N;
            for (uint32_t j = 0; j < N; j++) c[j] += a * (double)brow[j];
        }
    }
}

/* Selected GEMM outputs, one by one (for checks at sizes where the whole
 * product is too slow): out[t] = C[ii[t]][jj[t]]. */
void oracle_gemm_f64_entries(const float *A, const float *B, uint32_t N, uint32_t K, const uint32_t *ii,
                             const uint32_t *jj, uint64_t count, double *out) {
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < (int64_t)count; t++) {
        double acc = 0.0;
        for (uint32_t k = 0; k < K; k++)
            acc += (double)A[(uint64_t)ii[t] * K + k] * (double)B[(uint64_t)k * N + jj[t]];
        out[t] = acc;
    }
}
