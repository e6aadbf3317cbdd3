"""Pins of the CPU oracle against facts that do not come from the oracle:
closed forms, invariants, library routines the definition reduces to, the
paper's worked examples, and brute force on tiny inputs.  Each planted
mistake (a dropped barrier, a skipped read-before-write) must be caught.
"""

import json
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SEEDS = [0, 1, 2, 3, 0xDEADBEEF, 77, 1234567, 99]


# --------------------------------------------------------------------------
# input generator
# --------------------------------------------------------------------------

def test_splitmix64_reference_output():
    # Published SplitMix64: from state 0, the first output is the mix of
    # the golden-gamma increment, 0xE220A8397B1DCDAF.
    z = synth._mix(np.array([0x9E3779B97F4A7C15], dtype=np.uint64))
    assert int(z[0]) == 0xE220A8397B1DCDAF


def test_generators_ranges_and_counter_property():
    x = synth.uniform_int32(synth.SEED_REDUCE, 50000, -1000, 1000)
    assert x.min() == -1000 and x.max() == 1000
    # element i is regenerable on its own
    assert np.array_equal(synth.uniform_int32(synth.SEED_REDUCE, 100, -1000, 1000, start=1234), x[1234:1334])
    f = synth.uniform_f32(synth.SEED_JACOBI, 50000)
    assert f.min() >= 0.0 and f.max() < 1.0
    assert np.all(f * np.float32(2**24) == np.floor(f * np.float32(2**24)))


def test_zipf_generator_matches_its_distribution():
    # Bounded Zipf(1.1) over 256 ranks: H_{256,1.1} = 4.8421, p_0 = 0.2065.
    h = np.sum(1.0 / np.arange(1, 257) ** 1.1)
    assert abs(h - 4.8421) < 1e-3
    keys = synth.zipf_u32(synth.SEED_HIST, 1 << 20)
    assert keys.max() < 256
    p = np.bincount(keys, minlength=256) / keys.size
    assert abs(p[0] - 1.0 / h) < 3e-3
    assert abs(p[:8].sum() - 0.519) < 5e-3


@pytest.mark.parametrize("alpha,p0", [(0.0, 1 / 256), (2.0, 1 / (np.pi**2 / 6 - 1 / 256.5)), (3.0, 0.8319)])
def test_zipf_exponents_match_closed_forms(alpha, p0):
    # p_0 = 1 / H_{256,alpha}: 1/256 for the uniform law; H_{256,2} is
    # zeta(2) = pi^2/6 less its tail beyond 256, about 1/256.5; H_{256,3} =
    # 1.2020 (zeta(3) = 1.20206 less a tail below 1e-5).
    assert abs(1.0 / np.sum(1.0 / np.arange(1, 257) ** alpha) - p0) < 1e-4
    n = 1 << 20
    keys = synth.zipf_u32(synth.SEED_HIST, n, alpha)
    got = np.count_nonzero(keys == 0) / n
    assert abs(got - p0) < 5 * np.sqrt(p0 * (1 - p0) / n) + 1e-9


def test_bin_permutation_is_a_bijection_and_relabels_the_histogram():
    perm = synth.bin_permutation()
    assert sorted(perm.tolist()) == list(range(256))
    assert int(np.count_nonzero(perm == np.arange(256))) < 8  # not near the identity
    keys = synth.zipf_u32(5, 70001, 2.0) ^ (synth.uniform_u32(6, 70001) & np.uint32(0xFFFFFF00))
    moved = synth.permute_bins(keys, perm)
    assert np.array_equal(moved >> 8, keys >> 8)
    h, hm = oracle.hist256_u32(keys, 3, 64), oracle.hist256_u32(moved, 3, 64)
    assert np.array_equal(hm[perm], h)  # bin b's count moves to bin perm[b]


# --------------------------------------------------------------------------
# runtime: the paper's worked fetch examples
# --------------------------------------------------------------------------

def test_fetch_examples_from_the_paper():
    ex = json.load(open(os.path.join(GOLDEN, "runtime_fetch_examples.json")))["examples"]
    for e in ex:
        fetches, workers, bpf_used = oracle.pool_probe(e["grid"], e["pool"], e["bpf"])
        assert fetches == e["fetches"], e["what"]
        assert 1 <= workers <= e["max_workers"], e["what"]
        if "bpf_used" in e:
            assert bpf_used == e["bpf_used"], e["what"]


@pytest.mark.parametrize("grid,pool,bpf", [(1, 4, 0), (100, 7, 0), (100, 7, 3), (65536, 8, 0), (37, 8, 32)])
def test_fetch_count_is_ceil(grid, pool, bpf):
    fetches, workers, bpf_used = oracle.pool_probe(grid, pool, bpf)
    want_bpf = bpf if bpf else -(-grid // pool)
    assert bpf_used == want_bpf
    assert fetches == -(-grid // want_bpf)
    assert workers <= min(pool, fetches)


# --------------------------------------------------------------------------
# executor semantics: the paper's dynamic-shared-memory example
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 31, 64, 100, 1024])
def test_reverse_closed_form(n):
    d = np.arange(n, dtype=np.int32) * 3 - 7
    for seed in SEEDS[:4]:
        assert np.array_equal(oracle.reverse_i32(d, order_seed=seed), d[::-1])


def test_reverse_without_barrier_is_caught_by_poison():
    d = np.arange(256, dtype=np.int32)
    with pytest.raises(oracle.OracleError) as e:
        for seed in SEEDS:
            oracle.reverse_i32(d, order_seed=seed, skip_barrier=True)
    assert e.value.kind == "UNINIT"


def test_reverse_rejects_oversized_block():
    with pytest.raises(oracle.OracleError):
        oracle.reverse_i32(np.zeros(1025, np.int32))


# --------------------------------------------------------------------------
# REDUCE
# --------------------------------------------------------------------------

def _segments(n, grid):
    s = 4 * (-(-n // (4 * grid)))
    return [(min(b * s, n), min((b + 1) * s, n)) for b in range(grid)]


def test_reduce_config_shape_closed_form():
    n, grid, block = 1 << 20, 4096, 256
    x = synth.uniform_int32(synth.SEED_REDUCE, n, -1000, 1000)
    partials, total = oracle.reduce_i32(x, grid, block)
    assert total == int(x.astype(np.int64).sum())
    seg = x.reshape(grid, 256).astype(np.int64).sum(axis=1)
    assert np.array_equal(partials.astype(np.int64), seg)


def test_reduce_all_ones():
    partials, total = oracle.reduce_i32(np.ones(1 << 16, np.int32), 64, 256)
    assert total == 1 << 16
    assert np.all(partials == 1024)


@pytest.mark.parametrize("grid", [1, 2, 3])
@pytest.mark.parametrize("block", [32, 64])
@pytest.mark.parametrize("n", [1, 5, 127, 1000])
def test_reduce_brute_force_tiny(grid, block, n):
    rng = np.random.default_rng(n * 7 + grid)
    x = rng.integers(-(2**31), 2**31, n, dtype=np.int64).astype(np.int32)
    partials, total = oracle.reduce_i32(x, grid, block, order_seed=grid)
    acc = 0
    for v in x.tolist():
        acc = (acc + v) & 0xFFFFFFFF
    assert total & 0xFFFFFFFF == acc
    for b, (lo, hi) in enumerate(_segments(n, grid)):
        s = 0
        for v in x[lo:hi].tolist():
            s = (s + v) & 0xFFFFFFFF
        assert int(partials[b]) & 0xFFFFFFFF == s


def test_reduce_random_order_invariance_and_pool():
    x = synth.uniform_int32(7, 20000, -(2**30), 2**30)
    ref = oracle.reduce_i32(x, 37, 128)
    for seed in SEEDS:
        p, t = oracle.reduce_i32(x, 37, 128, order_seed=seed)
        assert t == ref[1] and np.array_equal(p, ref[0])
    for bpf in (0, 1, 5, 37):
        p, t = oracle.reduce_i32(x, 37, 128, pool=4, bpf=bpf)
        assert t == ref[1] and np.array_equal(p, ref[0])


def test_reduce_missing_barrier_is_caught():
    x = synth.uniform_int32(8, 4096, -1000, 1000)
    want = int(x.astype(np.int64).sum())
    caught = False
    for seed in SEEDS:
        try:
            _, t = oracle.reduce_i32(x, 4, 256, order_seed=seed, skip_barrier=True)
            caught |= t != want
        except oracle.OracleError:
            caught = True
    assert caught


# --------------------------------------------------------------------------
# SCAN
# --------------------------------------------------------------------------

def _check_scan_invariant(x, y):
    xu = x.view(np.uint32)
    yu = y.view(np.uint32)
    assert yu[0] == xu[0]
    assert np.array_equal((yu[1:] - yu[:-1]).astype(np.uint32), xu[1:])


@pytest.mark.parametrize("n,block,items", [(1, 32, 1), (33, 32, 1), (1000, 64, 4), (8191, 128, 3),
                                           (100000, 512, 16), (70000, 96, 7), (70001, 512, 64)])
def test_scan_invariant_and_all_ones(n, block, items):
    x = synth.uniform_int32(n, n, 0, 100)
    y = oracle.scan_i32(x, block=block, items=items)
    _check_scan_invariant(x, y)
    ones = oracle.scan_i32(np.ones(n, np.int32), block=block, items=items)
    assert np.array_equal(ones, np.arange(1, n + 1, dtype=np.int32))


def test_scan_wraps_modulo_2_32():
    x = np.full(5000, 2**30, np.int32)
    y = oracle.scan_i32(x, block=64, items=4)
    want = ((np.arange(1, 5001, dtype=np.uint64) * 2**30) % 2**32).astype(np.uint32).view(np.int32)
    assert np.array_equal(y, want)


def test_scan_random_order_and_pool():
    x = synth.uniform_int32(11, 30000, -(2**31), 2**31 - 1)
    ref = oracle.scan_i32(x, block=128, items=5)
    _check_scan_invariant(x, ref)
    for seed in SEEDS[:4]:
        assert np.array_equal(oracle.scan_i32(x, block=128, items=5, order_seed=seed), ref)
    assert np.array_equal(oracle.scan_i32(x, block=128, items=5, pool=3), ref)


def test_scan_total_matches_int64_sum():
    x = synth.uniform_int32(synth.SEED_SCAN, 1 << 18, 0, 100)
    y = oracle.scan_i32(x, block=512, items=16)
    assert int(y.view(np.uint32)[-1]) == int(x.astype(np.int64).sum()) % 2**32


# --------------------------------------------------------------------------
# HIST256
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n,grid,block", [(0, 1, 64), (1, 3, 32), (1000, 7, 64), (1 << 18, 128, 256)])
def test_hist_counts(n, grid, block):
    keys = synth.zipf_u32(synth.SEED_HIST, n) if n else np.zeros(0, np.uint32)
    keys = keys ^ (synth.uniform_u32(5, n) & np.uint32(0xFFFFFF00)) if n else keys
    h = oracle.hist256_u32(keys, grid, block)
    assert int(h.sum()) == n
    assert np.array_equal(h, np.bincount(keys & 255, minlength=256).astype(np.uint32))


def test_hist_order_and_pool_invariance():
    keys = synth.zipf_u32(3, 50000)
    ref = oracle.hist256_u32(keys, 64, 128)
    for seed in SEEDS[:4]:
        assert np.array_equal(oracle.hist256_u32(keys, 64, 128, order_seed=seed), ref)
    for bpf in (0, 1, 16):
        assert np.array_equal(oracle.hist256_u32(keys, 64, 128, pool=4, bpf=bpf), ref)


# --------------------------------------------------------------------------
# JACOBI5
# --------------------------------------------------------------------------

def _impulse_closed_form(t, dx, dy):
    """Value at offset (dx, dy) from a unit impulse after t sweeps of the
    4-neighbour average, far from the border: the 2-D walk probability
    4^-t * C(t, (t+x+y)/2) * C(t, (t+x-y)/2), zero on the wrong parity."""
    from math import comb

    if (t + dx + dy) % 2:
        return 0.0
    a = (t + dx + dy) // 2
    b = (t + dx - dy) // 2
    if a < 0 or b < 0 or a > t or b > t:
        return 0.0
    return comb(t, a) * comb(t, b) / 4.0**t


def test_jacobi_impulse_closed_form_bit_exact():
    n = 48
    u = np.zeros((n, n), np.float32)
    c = n // 2
    u[c, c] = 1.0
    want = np.zeros((n, n))
    for t in range(1, 15):
        u = oracle.jacobi5_f32(u, 16, 16, order_seed=t)
        for i in range(n):
            for j in range(n):
                want[i, j] = _impulse_closed_form(t, j - c, i - c)
        assert np.array_equal(u.astype(np.float64), want), t
    u64 = np.zeros((n, n), np.float32)
    u64[c, c] = 1.0
    assert np.array_equal(oracle.jacobi5_f64(u64, 14), want)
    assert np.array_equal(oracle.jacobi5_f32_sweeps(u64, 14).astype(np.float64), want)


def test_jacobi_linear_and_constant_fields_are_fixed_points():
    ny, nx = 37, 53
    i, j = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    lin = (i + 2 * j).astype(np.float32)
    assert np.array_equal(oracle.jacobi5_f32(lin, 16, 16), lin)
    assert np.array_equal(oracle.jacobi5_f32_sweeps(lin, 5), lin)
    const = np.full((ny, nx), 0.3, np.float32)
    assert np.array_equal(oracle.jacobi5_f32(const, 8, 4), const)
    assert np.array_equal(oracle.jacobi5_f64(lin, 3), lin.astype(np.float64))


@pytest.mark.parametrize("shape,bx,by", [((40, 40), 16, 16), ((33, 70), 16, 16), ((17, 5), 8, 4), ((64, 64), 32, 2)])
def test_jacobi_executor_matches_whole_grid_loop(shape, bx, by):
    u = synth.uniform_f32(synth.SEED_JACOBI, shape[0] * shape[1]).reshape(shape)
    one = oracle.jacobi5_f32(u, bx, by, order_seed=5)
    assert np.array_equal(one, oracle.jacobi5_f32_sweeps(u, 1))
    assert np.array_equal(one, oracle.jacobi5_f32(u, bx, by, pool=3))
    # border copied, interior by the definition in double: one fp32 sweep
    # is the correctly rounded value of the double sum of four fp32 values
    # up to two roundings
    ref = oracle.jacobi5_f64(u, 1)
    rel = np.abs(one - ref) / np.maximum(np.abs(ref), 1e-30)
    assert rel.max() <= 2.5 * 2.0**-24


def test_jacobi_f32_vs_f64_tolerance_small():
    u = synth.uniform_f32(synth.SEED_JACOBI, 256 * 256).reshape(256, 256)
    a = oracle.jacobi5_f32_sweeps(u, 100)
    b = oracle.jacobi5_f64(u, 100)
    assert (np.abs(a - b) / np.abs(b)).max() <= 1e-6


# --------------------------------------------------------------------------
# GEMM
# --------------------------------------------------------------------------

def test_gemm_integer_inputs_exact():
    rng = np.random.default_rng(5)
    M, N, K = 70, 130, 129
    A = rng.integers(-2, 3, (M, K)).astype(np.float32)
    B = rng.integers(-2, 3, (K, N)).astype(np.float32)
    want = A.astype(np.int64) @ B.astype(np.int64)
    assert np.array_equal(oracle.gemm_f32(A, B, order_seed=3).astype(np.int64), want)
    assert np.array_equal(oracle.gemm_f64(A, B).astype(np.int64), want)


def test_gemm_identity():
    A = synth.normal_f32(synth.SEED_GEMM, 65 * 77).reshape(65, 77)
    assert np.array_equal(oracle.gemm_f32(A, np.eye(77, dtype=np.float32)), A)


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (64, 64, 16), (65, 63, 17), (128, 96, 130), (3, 200, 5)])
def test_gemm_odd_shapes_within_summation_bound(M, N, K):
    A = synth.normal_f32(M * 1000 + K, M * K).reshape(M, K)
    B = synth.normal_f32(N * 1000 + K, K * N).reshape(K, N)
    c64 = A.astype(np.float64) @ B.astype(np.float64)
    mine64 = oracle.gemm_f64(A, B)
    assert np.abs(mine64 - c64).max() <= 1e-12 * max(1.0, np.abs(c64).max())
    c32 = oracle.gemm_f32(A, B, order_seed=1, pool=2)
    # any fp32 summation order: |dC| <= gamma_K * (|A||B|)
    gamma = K * 2.0**-24 / (1 - K * 2.0**-24)
    bound = gamma * (np.abs(A).astype(np.float64) @ np.abs(B).astype(np.float64))
    assert np.all(np.abs(c32 - c64) <= bound + 1e-30)


def test_gemm_dropped_k_term_is_outside_tolerance():
    # the GEMM gate (max-normalised error <= 1e-5 sqrt(K)) must reject a
    # product that misses one k term
    M = N = 64
    K = 256
    A = synth.normal_f32(1, M * K).reshape(M, K)
    B = synth.normal_f32(2, K * N).reshape(K, N)
    c64 = oracle.gemm_f64(A, B)
    bad = oracle.gemm_f64(A[:, 1:], B[1:, :])
    err = np.abs(bad - c64).max() / np.abs(c64).max()
    assert err > 1e-5 * np.sqrt(K) * 10
    good = oracle.gemm_f32(A, B)
    assert np.abs(good - c64).max() / np.abs(c64).max() <= 1e-5 * np.sqrt(K)


def test_gemm_entries_match_whole():
    A = synth.normal_f32(3, 40 * 50).reshape(40, 50)
    B = synth.normal_f32(4, 50 * 30).reshape(50, 30)
    whole = oracle.gemm_f64(A, B)
    ii = np.array([0, 39, 17, 5], np.uint32)
    jj = np.array([0, 29, 3, 11], np.uint32)
    assert np.array_equal(oracle.gemm_f64_entries(A, B, ii, jj), whole[ii, jj])


# --------------------------------------------------------------------------
# 32-lane warp operations
# --------------------------------------------------------------------------

def _warp_cases():
    nc = oracle.warptest_ncases()
    return nc, [oracle.warptest_case(c) for c in range(nc)]


def _run_warp(val, pred, grid=2, block=64, seed=0):
    return oracle.warptest(val, pred, grid, block, order_seed=seed)


def test_warp_shuffles_on_lane_ids_documented_examples():
    # values = lane id; CUDA's documented behaviour of each shuffle form
    total = 128
    val = np.arange(total, dtype=np.int32)
    pred = np.zeros(total, np.uint32)
    out = _run_warp(val, pred)
    nc, cases = _warp_cases()
    find = {cases[c]: c for c in range(768)}
    lane = np.arange(32)
    # shfl_up by 1 at full width: lane 0 keeps its value, others get lane-1
    up1 = out[find[("up", 1, 32)], :32]
    assert up1.tolist() == [0] + list(range(31))
    # shfl_down by 1 at width 8: last lane of each 8-group keeps its value
    dn = out[find[("down", 1, 8)], :32]
    assert dn.tolist() == [l if l % 8 == 7 else l + 1 for l in range(32)]
    # broadcast of lane 5 at full width, second warp sees its own lane 5
    assert np.all(out[find[("shfl", 5, 32)], :32] == 5)
    assert np.all(out[find[("shfl", 5, 32)], 32:64] == 37)
    # broadcast with width 4: lane 5 mod 4 = 1 of each group
    assert out[find[("shfl", 5, 4)], :8].tolist() == [1, 1, 1, 1, 5, 5, 5, 5]
    # xor 1 swaps neighbours
    assert out[find[("xor", 1, 32)], :4].tolist() == [1, 0, 3, 2]
    # width 1 is the identity for shfl, up and down
    for op in ("shfl", "up", "down"):
        for p in (0, 3, 31):
            assert np.array_equal(out[find[(op, p, 1)]], val)
    # xor may read lanes of earlier width groups but never later ones: at
    # width 1, lane l gets lane l^m when l^m < l, else keeps its own value
    assert out[find[("xor", 3, 1)], :4].tolist() == [0, 1, 1, 0]
    # at width 8, xor 8 reaches the previous 8-group only
    assert out[find[("xor", 8, 8)], :16].tolist() == list(range(8)) + list(range(8))
    # delta 0 is the identity
    for op in ("up", "down", "xor"):
        assert np.array_equal(out[find[(op, 0, 32)]], val)
    del lane


def test_warp_shfl_up_steps_give_segment_prefix_sums():
    # a Hillis-Steele scan built from shfl_up steps equals numpy's cumsum
    # within each width segment
    rng = np.random.default_rng(1)
    total = 64
    val = rng.integers(0, 1000, total).astype(np.int32)
    pred = np.zeros(total, np.uint32)
    nc, cases = _warp_cases()
    find = {cases[c]: c for c in range(768)}
    for w in (2, 4, 8, 16, 32):
        x = val.copy()
        d = 1
        while d < w:
            y = _run_warp(x, pred, 1, 64)[find[("up", d, w)]]
            lane = np.arange(total) % 32
            x = np.where((lane % w) >= d, x + y, x).astype(np.int32)
            d *= 2
        want = val.reshape(-1, w).cumsum(axis=1).reshape(-1)
        assert np.array_equal(x, want), w


def test_warp_xor_butterfly_gives_segment_sums_and_is_involution():
    rng = np.random.default_rng(2)
    total = 64
    val = rng.integers(-500, 500, total).astype(np.int32)
    pred = np.zeros(total, np.uint32)
    nc, cases = _warp_cases()
    find = {cases[c]: c for c in range(768)}
    for w in (2, 4, 8, 16, 32):
        x = val.copy()
        m = 1
        while m < w:
            x = (x + _run_warp(x, pred, 1, 64)[find[("xor", m, w)]]).astype(np.int32)
            m *= 2
        want = np.repeat(val.reshape(-1, w).sum(axis=1), w)
        assert np.array_equal(x, want), w
    out = _run_warp(val, pred, 1, 64)
    for m in range(32):
        once = out[find[("xor", m, 32)]]
        assert np.array_equal(_run_warp(once, pred, 1, 64)[find[("xor", m, 32)]], val)


def test_warp_up_then_down_restores_interior():
    total = 64
    val = (np.arange(total, dtype=np.int32) * 7919) % 10007
    pred = np.zeros(total, np.uint32)
    nc, cases = _warp_cases()
    find = {cases[c]: c for c in range(768)}
    for w in (4, 16, 32):
        for d in (1, 2, 3):
            if d >= w:
                continue
            up = _run_warp(val, pred, 1, 64)[find[("up", d, w)]]
            back = _run_warp(up, pred, 1, 64)[find[("down", d, w)]]
            lane = np.arange(total) % 32
            keep = (lane % w) < w - d
            assert np.array_equal(back[keep], val[keep])


def test_warp_votes_match_bit_packing():
    rng = np.random.default_rng(3)
    total = 128
    val = np.zeros(total, np.int32)
    pred = rng.integers(0, 2**32, total, dtype=np.uint64).astype(np.uint32)
    pred[64:96] = 0xFFFFFFFF  # third warp: every predicate bit set
    pred[96:128] &= np.uint32(0x7FFFFFFF)  # fourth warp: bit 31 never set
    out = _run_warp(val, pred, 2, 64, seed=9)
    nc, cases = _warp_cases()
    for c in range(768, 864):
        vote, bit, _ = cases[c]
        bits = ((pred >> np.uint32(bit)) & np.uint32(1)).astype(np.uint8)
        for w in range(4):
            lanes = bits[32 * w:32 * w + 32]
            mask = int(np.packbits(lanes[::-1]).view(">u4")[0])
            got = out[c, 32 * w:32 * w + 32].view(np.uint32)
            if vote == "ballot":
                assert np.all(got == mask)
            elif vote == "any":
                assert np.all(got == (1 if mask else 0))
            else:
                assert np.all(got == (1 if mask == 0xFFFFFFFF else 0))


def test_warp_constant_forms_equal_runtime_forms():
    total = 64
    val = np.arange(total, dtype=np.int32) * 3 + 1
    pred = np.zeros(total, np.uint32)
    out = _run_warp(val, pred, 1, 64, seed=4)
    nc, cases = _warp_cases()
    find = {cases[c]: c for c in range(768)}
    for c in range(864, nc):
        op, p, w = cases[c]
        assert np.array_equal(out[c], out[find[(op, p, w)]])


def test_warp_order_invariance():
    total = 256
    val = np.arange(total, dtype=np.int32)
    pred = (np.arange(total, dtype=np.uint32) * np.uint32(2654435761))
    ref = _run_warp(val, pred, 2, 128)
    for seed in SEEDS[:3]:
        assert np.array_equal(_run_warp(val, pred, 2, 128, seed=seed), ref)


# --------------------------------------------------------------------------
# COMPACT_I32: the plain definition, pinned by a list comprehension on small
# inputs, the extreme thresholds, and order and count identities.
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n,t", [(0, 0), (1, 0), (37, -5), (1000, 0), (4097, 900), (4097, -1001)])
def test_compact_brute_force(n, t):
    x = synth.uniform_int32(0xC0 + n, n, -1000, 1000)
    want = [int(v) for v in x if int(v) > t]
    got = oracle.compact_i32(x, t)
    assert got.dtype == np.int32 and got.tolist() == want


def test_compact_extreme_thresholds_and_identities():
    x = synth.uniform_int32(0xC1C, 1 << 16, -(2**31), 2**31 - 1)
    x[:3] = [-(2**31), 2**31 - 1, 0]
    assert oracle.compact_i32(x, 2**31 - 1).size == 0                 # nothing exceeds INT_MAX
    allbut = oracle.compact_i32(x, -(2**31))                           # everything but INT_MIN
    assert np.array_equal(allbut, x[x != -(2**31)])
    for t in (-(2**30), 0, 12345):
        y = oracle.compact_i32(x, t)
        assert y.size == int(np.count_nonzero(x > t))
        assert np.all(y > t)
        # the kept elements appear in input order: their positions in x increase
        pos = np.nonzero(x > t)[0]
        assert np.array_equal(x[pos], y)
