"""Parity of the HIP kernel classes with the CPU oracle, through the C ABI.

Integer classes must match bit for bit; the fp32 stencil must match the
oracle's fp32 run bit for bit and stay within 1e-6 relative of the FP64
run; the GEMM must stay within 1e-5*sqrt(K) max-normalised of the FP64
product.  Sizes span several tiles plus ragged tails; the workload sizes
are checked on sampled outputs or invariants.
"""

import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def spmd():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2206_07896_amd as m

    return m


def dev(a):
    import torch

    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).cuda()


def host(t, dtype=None):
    a = t.cpu().numpy()
    return a.view(dtype) if dtype is not None else a


# --------------------------------------------------------------------------
# REVERSE (the paper's example) and warp conformance
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 31, 64, 100, 1024])
def test_reverse(spmd, n):
    say("reverse", n)
    d = synth.uniform_int32(n, n, -(2**31), 2**31 - 1)
    t = dev(d)
    spmd.ops.reverse_i32(t)
    spmd.sync()
    assert np.array_equal(host(t), oracle.reverse_i32(d))


@pytest.mark.parametrize("grid,block", [(2, 64), (1, 32), (3, 96), (1, 1024)])
def test_warp_conformance(spmd, grid, block):
    say("warptest", grid, block)
    total = grid * block
    val = synth.uniform_int32(0x57A, total, -(2**31), 2**31 - 1)
    pred = synth.uniform_u32(0x57B, total)
    pred[:32] = 0xFFFFFFFF
    out = spmd.ops.warptest(dev(val), dev(pred), grid, block)
    spmd.sync()
    want = oracle.warptest(val, pred, grid, block)
    got = host(out)
    bad = np.argwhere(got != want)
    assert bad.size == 0, f"first mismatches (case, thread): {bad[:5].tolist()} -> {[oracle.warptest_case(int(c)) for c, _ in bad[:5]]}"


# --------------------------------------------------------------------------
# REDUCE
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n,grid,block", [(1, 1, 64), (1000, 3, 64), (12345, 37, 256), (1 << 16, 64, 1024),
                                          (100003, 4096, 128), (1 << 20, 4096, 256),
                                          # grids past the resident workgroups: 2, 4 and 8 logical blocks per
                                          # workgroup, with ragged and empty trailing segments
                                          (3 * (1 << 20) + 1, 8192, 256), ((1 << 20) + 3, 16384, 256),
                                          (500001, 8192, 64), (1 << 22, 65536, 512)])
def test_reduce(spmd, n, grid, block):
    say("reduce", n, grid, block)
    x = synth.uniform_int32(synth.SEED_REDUCE + n, n, -1000, 1000)
    want_p, want_t = oracle.reduce_i32(x, grid, block)
    xt = dev(x)
    ws = spmd.ops.workspace(spmd.REDUCE_I32, grid, block, n)
    for rep in range(3):  # the ticket counter re-arms itself
        p, out = spmd.ops.reduce_i32(xt, grid, block, ws=ws)
        spmd.sync()
        assert int(host(out)[0]) == want_t, rep
        assert np.array_equal(host(p), want_p), rep


def test_reduce_wrapping_and_unaligned(spmd):
    say("reduce wrap/unaligned")
    n = 50001
    x = synth.uniform_int32(99, n, -(2**31), 2**31 - 1)
    xt = dev(x)
    for grid in (13, 4096):  # one logical block per workgroup, then two
        want_p, want_t = oracle.reduce_i32(x[1:], grid, 256)
        p, out = spmd.ops.reduce_i32(xt[1:], grid, 256)  # 4-byte offset: scalar load path
        spmd.sync()
        assert int(host(out)[0]) == want_t, grid
        assert np.array_equal(host(p), want_p), grid


# --------------------------------------------------------------------------
# SCAN
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n,block,items", [(1, 64, 1), (100, 64, 1), (5000, 64, 4), (8193, 128, 8), (70001, 512, 16),
                                           (200000, 1024, 32), (123457, 256, 2), (300001, 512, 64),
                                           (65536 * 3 + 17, 256, 64), (40000, 512, 32),
                                           (65536 * 5 + 3, 512, 128), (100001, 256, 128), (1000, 64, 128),
                                           # 16384 and 32768 tiles of 64 and 128 elements, thousands of
                                           # blocks resident at once: look-backs that cross many windows
                                           (1 << 20, 64, 1), ((1 << 22) - 5, 64, 2)])
def test_scan(spmd, n, block, items):
    say("scan", n, block, items)
    x = synth.uniform_int32(synth.SEED_SCAN + n, n, -(2**31), 2**31 - 1)
    want = oracle.scan_i32(x, block=64, items=4)
    xt = dev(x)
    grid = spmd.ops.scan_grid(n, block, items)
    ws = spmd.ops.workspace(spmd.SCAN_I32, grid, block, n)
    for rep in range(3):  # epoch-tagged status words: no clearing between launches
        y = spmd.ops.scan_i32(xt, block, items, ws=ws)
        spmd.sync()
        got = host(y)
        assert np.array_equal(got, want), (rep, int(np.argmax(got != want)))


@pytest.mark.parametrize("block,items", [(512, 128), (256, 128), (512, 32)])
def test_scan_unaligned(spmd, block, items):
    """A 4-byte offset input and output: every tile takes the element-wise
    path (at 128 items its two passes, the second re-reading x), over many
    tiles and a ragged end, against the oracle."""
    import torch

    n = 3 * block * items * 7 + 11
    say("scan unaligned", n, block, items)
    x = synth.uniform_int32(0x5CA, n, -(2**31), 2**31 - 1)
    want = oracle.scan_i32(x, block=64, items=4)
    base = torch.zeros(n + 1, dtype=torch.int32, device="cuda")
    base[1:] = dev(x)
    out = torch.full((n + 1,), 7, dtype=torch.int32, device="cuda")
    spmd.ops.scan_i32(base[1:], block, items, y=out[1:])
    spmd.sync()
    got = host(out)
    assert got[0] == 7
    assert np.array_equal(got[1:], want), int(np.argmax(got[1:] != want))


@pytest.mark.parametrize("items", [16, 32, 64, 128])
def test_scan_workload_size(spmd, items):
    """2^26 int32 U[0, 100] at blockDim 512 -- at 128 items the measured
    step's launch (1024 tiles over the resident blocks, one per CU, so every
    block loops over several tiles), launched as the step does: twice on one workspace,
    into two outputs.  Checked over all 2^26 elements by the complete
    invariant (y[0] = x[0], y[i] - y[i-1] = x[i] mod 2^32) and against the
    oracle on a 2^20 prefix."""
    import torch

    n = 1 << 26
    say("scan 2^26 block 512 items", items)
    x = synth.uniform_int32(synth.SEED_SCAN, n, 0, 100)
    xt = dev(x)
    ws = spmd.ops.workspace(spmd.SCAN_I32, spmd.ops.scan_grid(n, 512, items), 512, n)
    ys = [torch.empty_like(xt) for _ in range(2)]
    for y in ys:
        spmd.ops.scan_i32(xt, 512, items, y=y, ws=ws)
    spmd.sync()
    xu = x.view(np.uint32)
    # a prefix of the scan is the scan of the prefix, whatever the launch shape
    # (the oracle's executor holds at most 64 items per thread)
    want_prefix = oracle.scan_i32(x[:1 << 20], 512, min(items, 64))
    for rep, y in enumerate(ys):
        got = host(y).view(np.uint32)
        assert got[0] == xu[0], rep
        bad = np.flatnonzero((got[1:] - got[:-1]).astype(np.uint32) != xu[1:])
        assert bad.size == 0, (rep, bad[:5] + 1)
        assert int(got[-1]) == int(x.astype(np.int64).sum()) % 2**32, rep
        assert np.array_equal(got[:1 << 20].view(np.int32), want_prefix), rep


@pytest.mark.parametrize("lg", [28, 30])
def test_scan_large_sizes(spmd, lg):
    """The measured step's launch shape (512 x 128) on 2^28 and 2^30 int32
    U[0, 100] generated on the device (the host generator's stream, which
    test_device_generator_matches_host pins): 16 and 64 tiles per persistent
    block.  Checked over every element on the device by the complete
    invariant, the last element by the closed form (the sum mod 2^32), and a
    2^20 prefix against the oracle."""
    import torch

    n = 1 << lg
    say("scan", f"2^{lg}", "block 512 items 128")
    xt = torch.empty(n, dtype=torch.int32, device="cuda")
    spmd.batch.synth_uniform_i32(xt, synth.SEED_SCAN, 0, 100)
    y = spmd.ops.scan_i32(xt, 512, 128)
    spmd.sync()
    assert int(y[0].item()) == int(xt[0].item())
    assert torch.equal(y[1:] - y[:-1], xt[1:])  # int32 arithmetic wraps: mod 2^32
    assert int(y[-1].item()) % 2**32 == int(xt.sum(dtype=torch.int64).item()) % 2**32
    x_prefix = synth.uniform_int32(synth.SEED_SCAN, 1 << 20, 0, 100)
    assert np.array_equal(host(y[: 1 << 20]), oracle.scan_i32(x_prefix, 512, 64))
    del xt, y
    torch.cuda.empty_cache()


# --------------------------------------------------------------------------
# HIST256
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n,grid,block", [(0, 4, 64), (1, 1, 64), (999, 3, 128), (100003, 64, 256),
                                          (1 << 20, 1024, 512), (777777, 5, 1024)])
def test_hist(spmd, n, grid, block):
    say("hist", n, grid, block)
    keys = synth.zipf_u32(synth.SEED_HIST + n, n) if n else np.zeros(0, np.uint32)
    if n:
        keys = keys ^ (synth.uniform_u32(3, n) & np.uint32(0xFFFFFF00))
    want = oracle.hist256_u32(keys, grid, block)
    kt = dev(keys) if n else dev(np.zeros(4, np.uint32))[:0]
    for rep in range(2):  # the histogram is overwritten, not accumulated
        h = spmd.ops.hist256_u32(kt, grid, block)
        spmd.sync()
        assert np.array_equal(host(h, np.uint32), want), rep


def test_launch_timed(spmd):
    """spmd_launch_timed gives spmd_launch's results; its event span, bound
    to the launch's first and last kernel dispatch (the histogram launch has
    two: clear, then count), is positive and lies inside a pair of events
    recorded around the calls, as does the span to a launch that binds its
    stop event alone; a launch with nothing to do records its events
    together; a refused launch raises."""
    import torch

    n = (1 << 20) + 77
    x = synth.uniform_int32(synth.SEED_SCAN + 11, n, -(2**31), 2**31 - 1)
    keys = synth.zipf_u32(synth.SEED_HIST + 11, n)
    want = oracle.scan_i32(x, block=64, items=4)
    want_h = oracle.hist256_u32(keys, 256, 1024)
    xt, kt = dev(x), dev(keys)
    for rep in range(3):
        say("launch_timed scan 512x16 and hist 256x1024", n, rep)
        ev = spmd.timing_events(5)
        o0, o1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        o0.record()
        y = spmd.ops.scan_i32(xt, 512, 16, events=ev[0:2])
        h = spmd.ops.hist256_u32(kt, 256, 1024, events=ev[2:4])
        y2 = spmd.ops.scan_i32(xt, 512, 16, events=(None, ev[4]))  # stop event only
        o1.record()
        o1.synchronize()
        spmd.sync()
        assert np.array_equal(host(y), want) and np.array_equal(host(y2), want)
        assert np.array_equal(host(h, np.uint32), want_h)
        t_scan, t_hist, t_out = ev[0].elapsed_time(ev[1]), ev[2].elapsed_time(ev[3]), o0.elapsed_time(o1)
        t_scan2 = ev[3].elapsed_time(ev[4])  # from the histogram's end to the second scan's end
        assert t_scan > 0 and t_hist > 0 and t_scan2 > 0, (t_scan, t_hist, t_scan2)
        assert t_scan + t_hist + t_scan2 <= t_out + 0.002, (t_scan, t_hist, t_scan2, t_out)
    say("launch_timed: empty scan, refused histogram")
    ev = spmd.timing_events(2)
    empty = torch.zeros(0, dtype=torch.int32, device="cuda")
    spmd.ops.scan_i32(empty, 512, 16, events=ev)
    ev[1].synchronize()
    assert ev[0].elapsed_time(ev[1]) >= 0
    with pytest.raises(spmd.SpmdError):
        spmd.ops.hist256_u32(kt, 256, 2048, events=spmd.timing_events(2))
    spmd.sync()


def skewed_keys(n, alpha, perm, seed):
    """Bounded Zipf(alpha) bins (or every key in bin 7 for alpha "one"),
    optionally through the seeded bin permutation, random upper bits."""
    upper = synth.uniform_u32(seed + 1, n) & np.uint32(0xFFFFFF00)
    if alpha == "one":
        return upper | np.uint32(7)
    keys = synth.zipf_u32(seed, n, alpha) | upper
    return synth.permute_bins(keys, synth.bin_permutation()) if perm else keys


@pytest.mark.parametrize("alpha,perm", [(0.0, False), (1.1, True), (1.5, False), (2.0, True), (3.0, False),
                                        ("one", False)])
@pytest.mark.parametrize("n,grid,block,offset", [((1 << 20) + 13, 256, 1024, 0), (300007, 7, 64, 1),
                                                 (1 << 16, 1024, 512, 0), (4099, 2, 256, 0)])
def test_hist_skew(spmd, alpha, perm, n, grid, block, offset):
    """Contention: skewed and one-bin keys, hot bins in place or permuted,
    16-byte aligned (vote path) and offset by one key (plain path)."""
    say("hist skew", alpha, perm, n, grid, block, offset)
    keys = skewed_keys(n + offset, alpha, perm, 0x51 + n)
    want = oracle.hist256_u32(keys[offset:], grid, block)
    h = spmd.ops.hist256_u32(dev(keys)[offset:], grid, block)
    spmd.sync()
    assert np.array_equal(host(h, np.uint32), want)


def test_hist_skew_workload_size(spmd):
    n = 1 << 27
    say("hist 2^27 zipf3 permuted, 256 x 1024")
    keys = skewed_keys(n, 3.0, True, synth.SEED_HIST)
    h = spmd.ops.hist256_u32(dev(keys), 256, 1024)
    spmd.sync()
    assert np.array_equal(host(h, np.uint32), oracle.hist256_u32(keys, 256, 1024, pool=16))


def test_hist_workload_size(spmd):
    n = 1 << 27
    say("hist 2^27 zipf")
    keys = synth.zipf_u32(synth.SEED_HIST, n)
    h = spmd.ops.hist256_u32(dev(keys), 1024, 512)
    spmd.sync()
    got = host(h, np.uint32)
    assert int(got.astype(np.int64).sum()) == n
    assert np.array_equal(got, oracle.hist256_u32(keys, 1024, 512, pool=16))


# --------------------------------------------------------------------------
# JACOBI5
# --------------------------------------------------------------------------

SHAPES = [(16, 16), (32, 8), (64, 4), (64, 8), (128, 2), (128, 4), (256, 1)]


@pytest.mark.parametrize("block", SHAPES)
@pytest.mark.parametrize("cells", [1, 4])
def test_jacobi_one_sweep(spmd, block, cells):
    # Block rows of 4 to 64 rows run 256 columns per workgroup: nx % 4 == 0 with aligned rows
    # takes the 16-byte form, any other nx the general-width form (four columns 64 apart);
    # block rows of 1 or 2 rows take the scalar body.
    # degenerate grids last: one row or column, or two (every cell a border cell, copied)
    for (ny, nx) in [(33, 70), (130, 257), (3, 3), (33, 68), (130, 520), (5, 4), (64, 260),
                     (1, 1), (1, 300), (300, 1), (2, 2), (2, 513), (1, 4), (2, 260)]:
        say("jacobi", ny, nx, block, cells)
        u = synth.uniform_f32(synth.SEED_JACOBI + nx, ny * nx).reshape(ny, nx)
        want = oracle.jacobi5_f32(u, 16, 16)
        got = host(spmd.ops.jacobi5_f32(dev(u), block=block, cells=cells))
        spmd.sync()
        assert np.array_equal(got, want)


def test_jacobi_misaligned_rows(spmd):
    """nx a multiple of 4 but the grid one float into its buffer: rows are
    not 16-byte aligned, so the general-width form runs."""
    import torch

    ny, nx = 70, 260
    say("jacobi misaligned rows", ny, nx)
    u = synth.uniform_f32(77, ny * nx).reshape(ny, nx)
    buf = torch.zeros(ny * nx + 1, dtype=torch.float32, device="cuda")
    buf[1:] = dev(u).reshape(-1)
    out = torch.zeros(ny * nx + 1, dtype=torch.float32, device="cuda")
    spmd.ops.jacobi5_f32(buf[1:].view(ny, nx), out=out[1:].view(ny, nx), block=(64, 4), cells=4)
    spmd.sync()
    assert np.array_equal(host(out[1:]).reshape(ny, nx), oracle.jacobi5_f32(u, 16, 16))


@pytest.mark.parametrize("nx", [517, 516])
def test_jacobi_sweeps_bit_exact(spmd, nx):
    ny = 300
    say("jacobi 25 sweeps", ny, nx)
    u = synth.uniform_f32(5, ny * nx).reshape(ny, nx)
    got = host(spmd.ops.jacobi5_sweeps(dev(u), 25, block=(64, 4), cells=4))
    spmd.sync()
    assert np.array_equal(got, oracle.jacobi5_f32_sweeps(u, 25))


def test_jacobi_workload_size(spmd):
    n, sweeps = 8192, 100
    say("jacobi 8192^2 x 100, 16x16 blocks")
    u = synth.uniform_f32(synth.SEED_JACOBI, n * n).reshape(n, n)
    got = host(spmd.ops.jacobi5_sweeps(dev(u), sweeps, block=(16, 16), cells=1))
    spmd.sync()
    ref64 = oracle.jacobi5_f64(u, sweeps)
    rel = np.abs(got.astype(np.float64) - ref64) / np.abs(ref64)
    assert rel.max() <= 1e-6, rel.max()
    want = oracle.jacobi5_f32_sweeps(u, sweeps)
    assert np.array_equal(got, want)
    for per in (4, 8):  # the fused-sweep class: 25 launches of 4, or 12 of 8 and one of 4
        say("jacobi 8192^2 x 100 fused", per)
        got = host(spmd.ops.jacobi5t_sweeps(dev(u), sweeps, per_launch=per))
        spmd.sync()
        assert np.array_equal(got, want), per


# --------------------------------------------------------------------------
# JACOBI5T: fused sweeps
# --------------------------------------------------------------------------

@pytest.mark.parametrize("sweeps", [1, 2, 3, 4, 5, 8])
def test_jacobi_fused_bit_exact(spmd, sweeps):
    """S sweeps in one launch equal S sweeps of the oracle, on grids that
    are smaller than, equal to and ragged against the 128 x 64 tile."""
    for (ny, nx) in [(1, 4), (2, 8), (3, 4), (5, 12), (64, 128), (65, 132), (131, 516), (200, 260), (63, 1028)]:
        say("jacobi fused", sweeps, ny, nx)
        u = synth.uniform_f32(0x5EED + nx * 7 + ny, ny * nx).reshape(ny, nx)
        got = host(spmd.ops.jacobi5t_f32(dev(u), sweeps))
        spmd.sync()
        assert np.array_equal(got, oracle.jacobi5_f32_sweeps(u, sweeps)), (ny, nx)


def test_jacobi_fused_chain_and_closed_form(spmd):
    """27 sweeps as 8 + 8 + 8 + 3 fused launches against the oracle, and the
    linear field u = i + 2j, a fixed point of the stencil, through 8."""
    ny, nx = 300, 1028
    u = synth.uniform_f32(0xF00D, ny * nx).reshape(ny, nx)
    got = host(spmd.ops.jacobi5t_sweeps(dev(u), 27, per_launch=8))
    spmd.sync()
    assert np.array_equal(got, oracle.jacobi5_f32_sweeps(u, 27))
    i, j = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    lin = (i + 2 * j).astype(np.float32)
    got = host(spmd.ops.jacobi5t_f32(dev(lin), 8))
    spmd.sync()
    assert np.array_equal(got, lin)


def test_jacobi_fused_rejects_bad_launches(spmd):
    import torch

    u = dev(np.zeros((64, 128), np.float32))
    v = torch.empty_like(u)
    ok = ((1, 1, 1), (256, 1, 1))
    for args, grid, block, kind in [([u, v, 128, 64, 0], *ok, "ARGS"), ([u, v, 128, 64, 9], *ok, "ARGS"),
                                    ([u, v, 126, 64, 2], *ok, "ARGS"), ([u, u, 128, 64, 2], *ok, "ARGS"),
                                    ([u, v, 128, 64, 2], (1, 1, 1), (128, 1, 1), "INVALID_DIM"),
                                    ([u, v, 256, 32, 2], *ok, "INVALID_DIM"),  # 248 columns per tile
                                    ([u.view(-1)[1:], v, 124, 64, 2], *ok, "ARGS")]:
        with pytest.raises(spmd.SpmdError) as e:
            spmd.launch(spmd.JACOBI5T_F32, grid, block, 0, args)
        assert e.value.kind == kind, (args[2:], grid, block)


# --------------------------------------------------------------------------
# GEMM
# --------------------------------------------------------------------------

def _gemm_gate(C, c64, K):
    return np.abs(C.astype(np.float64) - c64).max() / np.abs(c64).max() <= 1e-5 * np.sqrt(K)


@pytest.mark.parametrize("tile", [64, 128, 256])
@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (64, 64, 16), (65, 63, 17), (128, 96, 130), (3, 200, 5), (257, 130, 64),
                                   (512, 512, 512),
                                   # 16-byte rows (N, K multiples of 4): the direct-to-LDS form, with
                                   # K below one slice, K tails of 4 / 8 / 12, slice counts on both
                                   # sides of its pipeline's main loop, and rows / columns past C
                                   (1, 4, 4), (33, 68, 8), (100, 124, 12), (64, 64, 32), (70, 260, 48),
                                   (130, 132, 96), (129, 256, 112), (200, 196, 116), (256, 256, 200),
                                   (300, 300, 1028)])
def test_gemm_shapes(spmd, tile, M, N, K):
    say("gemm", M, N, K, tile)
    A = synth.normal_f32(M * 7 + K, M * K).reshape(M, K)
    B = synth.normal_f32(N * 11 + K, K * N).reshape(K, N)
    C = host(spmd.ops.gemm_f32(dev(A), dev(B), tile=tile))
    spmd.sync()
    c64 = oracle.gemm_f64(A, B)
    assert _gemm_gate(C, c64, K)
    gamma = K * 2.0**-24 / (1 - K * 2.0**-24)
    bound = gamma * (np.abs(A).astype(np.float64) @ np.abs(B).astype(np.float64))
    assert np.all(np.abs(C - c64) <= bound + 1e-30)


@pytest.mark.parametrize("tile", [64, 128, 256])
def test_gemm_exact_cases(spmd, tile):
    say("gemm exact", tile)
    rng = np.random.default_rng(7)
    M, N, K = 200, 136, 300
    A = rng.integers(-2, 3, (M, K)).astype(np.float32)
    B = rng.integers(-2, 3, (K, N)).astype(np.float32)
    C = host(spmd.ops.gemm_f32(dev(A), dev(B), tile=tile))
    assert np.array_equal(C.astype(np.int64), A.astype(np.int64) @ B.astype(np.int64))
    A2 = synth.normal_f32(1, 100 * 77).reshape(100, 77)
    C2 = host(spmd.ops.gemm_f32(dev(A2), dev(np.eye(77, dtype=np.float32)), tile=tile))
    spmd.sync()
    assert np.array_equal(C2, A2)


@pytest.mark.parametrize("tile", [64, 128, 256])
def test_gemm_grid_larger_than_c(spmd, tile):
    """A grid with more tiles than C needs: the extra blocks store nothing
    (C sits between guard words that must stay as they were)."""
    import torch

    M, N, K = 150, 100, 68
    say("gemm oversized grid", tile)
    A = synth.normal_f32(5, M * K).reshape(M, K)
    B = synth.normal_f32(6, K * N).reshape(K, N)
    guard = 1 << 12
    buf = torch.full((M * N + 2 * guard,), 7.0, dtype=torch.float32, device="cuda")
    C = buf[guard:guard + M * N]
    grid = (-(-N // tile) + 3, -(-M // tile) + 2)
    spmd.launch(spmd.GEMM_F32, grid, 256, 0, [dev(A), dev(B), C, M, N, K])
    spmd.sync()
    got = host(buf)
    assert np.all(got[:guard] == 7.0) and np.all(got[guard + M * N:] == 7.0)
    assert _gemm_gate(got[guard:guard + M * N].reshape(M, N), oracle.gemm_f64(A, B), K)


@pytest.mark.parametrize("tile", [64, 128, 256])
def test_gemm_workload_size(spmd, tile):
    n = 4096
    say("gemm 4096^3", tile)
    A = synth.normal_f32(synth.SEED_GEMM, n * n).reshape(n, n)
    B = synth.normal_f32(synth.SEED_GEMM + 1, n * n).reshape(n, n)
    C = host(spmd.ops.gemm_f32(dev(A), dev(B), tile=tile))
    spmd.sync()
    rng = np.random.default_rng(3)
    rows = rng.choice(n, 4, replace=False)
    ii = np.concatenate([np.repeat(rows, n), rng.integers(0, n, 4096)]).astype(np.uint32)
    jj = np.concatenate([np.tile(np.arange(n), 4), rng.integers(0, n, 4096)]).astype(np.uint32)
    c64 = oracle.gemm_f64_entries(A, B, ii, jj)
    d = np.abs(C[ii, jj].astype(np.float64) - c64)
    assert d.max() / np.abs(c64).max() <= 1e-5 * np.sqrt(n)


def test_scan_forms_share_a_workspace(spmd):
    """Every launch shape (tile size, tile count, resident block count)
    advances the same epoch and re-arms the ticket at its own last draw, so
    alternating shapes on one workspace must stay exact."""
    n = 300_007
    say("scan alternating forms", n)
    x = synth.uniform_int32(17, n, -(2**31), 2**31 - 1)
    want = oracle.scan_i32(x, 64, 4)
    xt = dev(x)
    grid_max = spmd.ops.scan_grid(n, 64, 1)
    ws = spmd.ops.workspace(spmd.SCAN_I32, grid_max, 64, n)
    for block, items in [(64, 1), (256, 8), (64, 2), (512, 16), (128, 4), (1024, 32), (64, 1)]:
        y = spmd.ops.scan_i32(xt, block, items, ws=ws)
        spmd.sync()
        assert np.array_equal(host(y), want), (block, items)


def test_scan_graph_replays(spmd):
    """Three scans of different shapes on one workspace, captured in a graph:
    replays interleaved with eager scans on the same workspace and host
    synchronisations, every replay exact."""
    import torch

    n = 200_003
    say("scan graph replays", n)
    x = synth.uniform_int32(23, n, -(2**31), 2**31 - 1)
    want = oracle.scan_i32(x, 64, 4)
    xt = dev(x)
    ws = spmd.ops.workspace(spmd.SCAN_I32, spmd.ops.scan_grid(n, 64, 1), 64, n)
    ys = [torch.empty_like(xt) for _ in range(3)]
    shapes = [(512, 64), (256, 8), (1024, 32)]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up outside the capture
        for (b, i), y in zip(shapes, ys):
            spmd.ops.scan_i32(xt, b, i, y=y, ws=ws)
    torch.cuda.current_stream().wait_stream(side)
    spmd.sync()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for (b, i), y in zip(shapes, ys):
            spmd.ops.scan_i32(xt, b, i, y=y, ws=ws)
    for rep in range(3):
        for y in ys:
            y.fill_(0)
        g.replay()
        spmd.sync()
        for y in ys:
            assert np.array_equal(host(y), want), rep
        e = spmd.ops.scan_i32(xt, 128, 16, ws=ws)  # eager work between replays
        spmd.sync()
        assert np.array_equal(host(e), want), rep


def test_maximum_size_closed_forms(spmd):
    """n = 2^32 - 1, the largest count a uint32 argument holds (16 GiB per
    array): scan of ones is y[i] = i + 1 mod 2^32, the sum of ones is
    2^32 - 1 (int32 -1), every key in one bin fills it with 2^32 - 1, and
    compaction keeps everything.  Element offsets pass 2^31 and 2^32 - 1, so
    any 32-bit index in a kernel would show.  Checked on the device at 2^20
    random positions plus both ends and the 2^31 boundary."""
    import torch

    n = 2**32 - 1
    say("maximum size", n)
    g = torch.Generator(device="cuda").manual_seed(5)
    idx = torch.randint(0, n, (1 << 20,), device="cuda", generator=g, dtype=torch.int64)
    idx = torch.cat([idx, torch.tensor([0, 1, 2**31 - 2, 2**31 - 1, 2**31, 2**31 + 1, n - 2, n - 1],
                                       device="cuda")])
    as_i32 = lambda v: (v & 0xFFFFFFFF).to(torch.int32)  # noqa: E731 -- wrap to the int32 bit pattern
    x = torch.ones(n, dtype=torch.int32, device="cuda")
    y = spmd.ops.scan_i32(x, 1024, 32)
    spmd.sync()
    assert bool(torch.equal(y[idx], as_i32(idx + 1)))
    del y
    torch.cuda.empty_cache()
    _, out = spmd.ops.reduce_i32(x, 4096, 256)
    spmd.sync()
    assert int(out.item()) == -1
    yc, cnt = spmd.ops.compact_i32(x, 0, 1024, 32)
    spmd.sync()
    assert int(cnt.item()) == -1  # 2^32 - 1 as int32
    assert bool(torch.equal(yc[idx], x[idx]))
    del yc
    torch.cuda.empty_cache()
    x.fill_(5 + 256 * 7)
    h = spmd.ops.hist256_u32(x, 256, 1024)
    spmd.sync()
    hh = host(h, np.uint32)
    assert int(hh[5]) == n and int(hh.astype(np.int64).sum()) == n
    del x
    torch.cuda.empty_cache()


# --------------------------------------------------------------------------
# COMPACT_I32 (warp vote: ballot + popc)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n,block,items,t", [(1, 64, 1, 0), (100, 64, 1, 0), (5000, 64, 4, -1),
                                             (8193, 128, 8, 500), (70001, 256, 16, 0),
                                             (200000, 1024, 32, -900), (123457, 512, 2, 999),
                                             (4096 * 16 * 3, 256, 16, 0), (300001, 512, 64, 0),
                                             (65536 * 3 + 17, 256, 64, -3), (1 << 20, 64, 1, 0)])
def test_compact(spmd, n, block, items, t):
    import torch

    say("compact", n, block, items, t)
    x = synth.uniform_int32(0xC0 + n, n, -1000, 1000)
    want = oracle.compact_i32(x, t)
    xt = dev(x)
    grid = spmd.ops.compact_grid(n, block, items)
    ws = spmd.ops.workspace(spmd.COMPACT_I32, grid, block, n)
    y = torch.full((n,), 7, dtype=torch.int32, device="cuda")
    for rep in range(3):  # the workspace is reused without clearing
        count = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        spmd.ops.compact_i32(xt, t, block, items, y=y, count=count, ws=ws)
        spmd.sync()
        m = int(count.item())
        got = host(y)
        assert m == want.size, (rep, m, want.size)
        assert np.array_equal(got[:m], want), rep
        assert np.all(got[m:] == (7 if rep == 0 else got[m:]))  # untouched beyond m


def test_compact_edges(spmd):
    import torch

    say("compact edges")
    n = 1 << 16
    x = synth.uniform_int32(0xC1D, n, -(2**31), 2**31 - 1)
    x[:2] = [-(2**31), 2**31 - 1]
    xt = dev(x)
    for t in (2**31 - 1, -(2**31), 0):
        y, count = spmd.ops.compact_i32(xt, t)
        spmd.sync()
        want = oracle.compact_i32(x, t)
        assert int(count.item()) == want.size and np.array_equal(host(y)[: want.size], want)
    # unaligned input (the per-element path for every tile) and empty input
    xu = torch.from_numpy(x[: n - 3].copy()).cuda()
    base = torch.zeros(n + 1, dtype=torch.int32, device="cuda")
    base[1:n - 2] = xu
    y, count = spmd.ops.compact_i32(base[1:n - 2], 0)
    spmd.sync()
    want = oracle.compact_i32(x[: n - 3], 0)
    assert int(count.item()) == want.size and np.array_equal(host(y)[: want.size], want)
    empty = torch.empty(0, dtype=torch.int32, device="cuda")
    y, count = spmd.ops.compact_i32(empty, 0)
    spmd.sync()
    assert int(count.item()) == 0


@pytest.mark.parametrize("block,items", [(256, 16), (1024, 32)])
def test_compact_many_tiles_per_block(spmd, block, items):
    """Thousands of tiles, so each persistent block runs its two-tile
    pipeline many times: an unaligned input (every tile takes the
    element-wise passes) and an aligned one with a ragged tail (row tiles,
    then a partial last tile in the same pipeline), against the oracle."""
    import torch

    n = (1 << 22) + 777
    x = synth.uniform_int32(0xC1E, n + 1, -1000, 1000)
    base = dev(x)
    for off in (1, 0):
        say("compact many tiles", block, items, "offset", off)
        xt = base[off:off + n]
        want = oracle.compact_i32(x[off:off + n], 0)
        y, count = spmd.ops.compact_i32(xt, 0, block, items)
        spmd.sync()
        m = int(count.item())
        assert m == want.size, (off, m, want.size)
        bad = np.flatnonzero(host(y)[:m] != want)
        assert bad.size == 0, (off, bad[:5])


@pytest.mark.parametrize("block,items", [(256, 16), (1024, 32), (512, 32)])
def test_compact_workload_size(spmd, block, items):
    """2^26 int32 U[-1000, 1000], t = 0, element by element against the
    oracle -- at 1024 x 32 and 512 x 32 the measured launches, run as the
    measurement does: twice on one workspace, with the input rotated over
    two copies and one output reused."""
    import torch

    say("compact 2^26, t = 0", block, items)
    n = 1 << 26
    x = synth.uniform_int32(synth.SEED_SCAN, n, -1000, 1000)
    xs = [dev(x), dev(x)]
    ws = spmd.ops.workspace(spmd.COMPACT_I32, spmd.ops.compact_grid(n, block, items), block, n)
    y = torch.full((n,), 7, dtype=torch.int32, device="cuda")
    want = oracle.compact_i32(x, 0)
    for rep in range(2):
        count = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        spmd.ops.compact_i32(xs[rep], 0, block, items, y=y, count=count, ws=ws)
        spmd.sync()
        m = int(count.item())
        assert m == want.size, (rep, m)
        got = host(y)
        bad = np.flatnonzero(got[:m] != want)
        assert bad.size == 0, (rep, bad[:5])
        assert np.all(got[m:] == 7), rep  # untouched beyond the count
