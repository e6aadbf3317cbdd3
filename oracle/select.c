/* Stream compaction -- TEST INFRASTRUCTURE ONLY: nothing on the product
 * path includes, links or calls this code.
 *
 * The plain definition of the COMPACT_I32 class, a database selection: the
 * elements of x strictly greater than t, in their input order, and how many
 * there are.  It stands for the filter operators of the GPU database
 * queries the paper covers (Section V-A, benchmark coverage), whose CUDA
 * kernels rest on warp vote and shuffle.
 */
#include <stdint.h>

int oracle_compact_i32(const int32_t *x, uint64_t n, int32_t t, int32_t *y, uint64_t *count) {
    uint64_t m = 0;
    for (uint64_t i = 0; i < n; i++)
        if (x[i] > t) y[m++] = x[i];
    *count = m;
    return 0;
}
