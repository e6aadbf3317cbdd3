/* spmd_synth.h -- seeded synthetic inputs generated on the device.
 *
 * Input generation only: nothing here is part of the kernel classes.  The
 * generator is counter-based SplitMix64 (Steele, Lea and Flood, "Fast
 * splittable pseudorandom number generators", OOPSLA 2014): for a stream
 * key K (the SplitMix64 mix of the seed) element i is
 *   h_i = mix(K + (i + 1) * 0x9E3779B97F4A7C15)   (mod 2^64)
 * with mix(z) = z ^= z >> 30, z *= 0xBF58476D1CE4E5B9, z ^= z >> 27,
 * z *= 0x94D049BB133111EB, z ^= z >> 31.  Derived values:
 *   uniform int32 in [lo, hi]: lo + (((h >> 32) * (hi - lo + 1)) >> 32)
 *   uniform fp32 in [0, 1):    (h >> 40) * 2^-24
 *   raw uint32:                h >> 32
 *   bounded Zipf key:          the number of entries of `cdf` (k ascending
 *                              doubles) that are <= u, u = (h >> 11) * 2^-53,
 *                              capped at k - 1.
 * Element i of the output is element start + i of the stream, so any range
 * can be generated on its own.  All calls are asynchronous on `stream`.
 */
#ifndef SPMD_SYNTH_H
#define SPMD_SYNTH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The stream key of a seed (one mix of the seed). */
uint64_t spmd_synth_key(uint64_t seed);

int spmd_synth_uniform_i32(int32_t* out, uint64_t count, uint64_t seed, uint64_t start, int32_t lo, int32_t hi,
                           void* stream);
int spmd_synth_uniform_f32(float* out, uint64_t count, uint64_t seed, uint64_t start, void* stream);
int spmd_synth_raw_u32(uint32_t* out, uint64_t count, uint64_t seed, uint64_t start, void* stream);
/* `cdf`: device array of k ascending doubles (the Zipf CDF), k <= 65536. */
int spmd_synth_zipf_u32(uint32_t* out, uint64_t count, uint64_t seed, uint64_t start, const double* cdf,
                        uint32_t k, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* SPMD_SYNTH_H */
