"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module holds no arithmetic of the kernel classes: it only turns a seed
and an element index into input values.  Both sides of every parity check
receive arrays produced here, so neither side ever derives its inputs from
the other.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014), used counter-style.  The stream for a seed
starts at state ``key = mix(seed)``; element ``i`` of the stream is the
SplitMix64 output after ``i + 1`` state increments::

    z   = key + (i + 1) * 0x9E3779B97F4A7C15          (mod 2^64)
    z   = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z   = (z ^ (z >> 27)) * 0x94D049BB133111EB
    h_i = z ^ (z >> 31)

so any element can be regenerated on its own (instances of a batch, sampled
checks at full size) without materialising the stream before it.

Derived distributions:

* integers uniform in ``[lo, hi]`` (inclusive): Lemire's multiply-shift
  without rejection, ``lo + (((h >> 32) * (hi - lo + 1)) >> 32)``;
* fp32 uniform in ``[0, 1)``: ``(h >> 40) * 2^-24`` (exactly representable);
* bounded Zipf(alpha) over ranks ``1..K``: inverse CDF in fp64 on
  ``u = (h >> 11) * 2^-53``; rank ``r`` becomes key ``r - 1``;
* N(0, 1): Box-Muller in fp64 from two stream elements (indices ``2i`` and
  ``2i + 1``), rounded to fp32;
* a seeded permutation of the 256 histogram bins (Fisher-Yates, swap
  partner of position ``j`` from 256 down to 2: Lemire's multiply-shift of
  element ``256 - j`` onto ``[0, j)``), so that a skewed law's hot bins land
  at scattered bins rather than 0, 1, 2, ...
"""

from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)

# Fixed seeds of the synthetic workloads.
SEED_REDUCE = 0xC1
SEED_SCAN = 0xC2A
SEED_HIST = 0xC2B
SEED_JACOBI = 0xC3A
SEED_GEMM = 0xC3B
SEED_BATCH = 0xC4
SEED_TRAIN = 0xC5
SEED_HELDOUT = 0xC5F
SEED_BIN_PERM = 0xC2C

_CHUNK = 1 << 22


def _mix(z: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
    return z ^ (z >> np.uint64(31))


def stream_key(seed: int) -> np.uint64:
    """Initial SplitMix64 state for ``seed``: one mixing round of the seed."""
    return _mix(np.array([seed & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64))[0]


def hashes(seed: int, start: int, count: int) -> np.ndarray:
    """Elements ``start .. start+count-1`` of the stream for ``seed`` (uint64)."""
    key = stream_key(seed)
    idx = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = key + idx * GAMMA
    return _mix(z)


def _chunked(count: int, fn, dtype) -> np.ndarray:
    out = np.empty(count, dtype=dtype)
    for s in range(0, count, _CHUNK):
        e = min(count, s + _CHUNK)
        out[s:e] = fn(s, e - s)
    return out


def uniform_int32(seed: int, count: int, lo: int, hi: int, start: int = 0) -> np.ndarray:
    """int32 uniform on the inclusive range [lo, hi] (Lemire, no rejection)."""
    span = np.uint64(hi - lo + 1)

    def fn(s, c):
        h = hashes(seed, start + s, c) >> np.uint64(32)
        with np.errstate(over="ignore"):
            v = (h * span) >> np.uint64(32)
        return (v.astype(np.int64) + lo).astype(np.int32)

    return _chunked(count, fn, np.int32)


def uniform_f32(seed: int, count: int, start: int = 0) -> np.ndarray:
    """fp32 uniform on [0, 1): the top 24 bits of each hash times 2^-24."""

    def fn(s, c):
        h = hashes(seed, start + s, c) >> np.uint64(40)
        return (h.astype(np.float64) * 2.0**-24).astype(np.float32)

    return _chunked(count, fn, np.float32)


def zipf_cdf(alpha: float, k: int) -> np.ndarray:
    """Cumulative probabilities of ranks 1..k for bounded Zipf(alpha), fp64."""
    w = 1.0 / np.power(np.arange(1, k + 1, dtype=np.float64), alpha)
    c = np.cumsum(w)
    return c / c[-1]


def zipf_u32(seed: int, count: int, alpha: float = 1.1, k: int = 256, start: int = 0) -> np.ndarray:
    """uint32 keys in [0, k): rank r of bounded Zipf(alpha) becomes key r-1."""
    cdf = zipf_cdf(alpha, k)

    def fn(s, c):
        u = (hashes(seed, start + s, c) >> np.uint64(11)).astype(np.float64) * 2.0**-53
        r = np.searchsorted(cdf, u, side="right")
        return np.minimum(r, k - 1).astype(np.uint32)

    return _chunked(count, fn, np.uint32)


def normal_f32(seed: int, count: int, start: int = 0) -> np.ndarray:
    """fp32 N(0,1) by Box-Muller (cosine branch) from hashes 2i and 2i+1."""

    def fn(s, c):
        h = hashes(seed, 2 * (start + s), 2 * c)
        u1 = ((h[0::2] >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0**-53
        u2 = (h[1::2] >> np.uint64(11)).astype(np.float64) * 2.0**-53
        z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
        return z.astype(np.float32)

    return _chunked(count, fn, np.float32)


def uniform_u32(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Raw uint32 words: the top 32 bits of each hash."""

    def fn(s, c):
        return (hashes(seed, start + s, c) >> np.uint64(32)).astype(np.uint32)

    return _chunked(count, fn, np.uint32)


def uniform_unit_f64(seed: int, count: int, start: int = 0) -> np.ndarray:
    """fp64 uniform on [0, 1): the top 53 bits of each hash times 2^-53."""
    return (hashes(seed, start, count) >> np.uint64(11)).astype(np.float64) * 2.0**-53


def bin_permutation(seed: int = SEED_BIN_PERM, k: int = 256) -> np.ndarray:
    """A permutation of ``0..k-1`` by Fisher-Yates from the seed's stream."""
    perm = np.arange(k, dtype=np.uint32)
    h = hashes(seed, 0, k)
    for j in range(k, 1, -1):
        r = int(((int(h[k - j]) >> 32) * j) >> 32)
        perm[j - 1], perm[r] = perm[r], perm[j - 1]
    return perm


def permute_bins(keys: np.ndarray, perm: np.ndarray) -> np.ndarray:
    """Keys with their low byte (the bin) sent through ``perm``."""
    keys = np.asarray(keys, dtype=np.uint32)
    return (keys & np.uint32(0xFFFFFF00)) | perm[keys & np.uint32(255)]
