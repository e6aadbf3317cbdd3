"""Completion and the device error word (spmd_sync, spmd_sync_timeout,
spmd_set_spin_limit), on the GPU.

Host-side behaviour of the paper's runtime: the host waits until the queue
has drained before it reads results (Section IV), and a barrier separates a
launch from work that reads its output (Section III-C1).  Here a sync waits
for the stream and then reports -- and clears -- the device's error word,
which a kernel sets when one of its bounded cross-block waits gives up.

No test makes a kernel fault or hang: the failure is forced from the host,
by a scan ticket that skips tile 0 (so tile 1's look-back waits for a tile
that is never drawn) under a spin limit of a few hundred polls, so every
wait ends within milliseconds and every kernel exits normally.
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

    assert torch.cuda.is_available()
    import paper_2206_07896_amd as m

    return m


def _scan_skipping_tile0(spmd, x, block, items, stream=None):
    """A scan whose ticket starts at 1 (epoch 0): tile 0 is never drawn, so
    the look-back of tile 1 (and of any tile that reaches back past it)
    waits for a status word that is never published and gives up at the
    spin limit.  The draws still end: tiles 1 .. G-1 and one terminating
    draw per block, the last of which re-arms the ticket."""
    import torch

    n = x.numel()
    grid = spmd.ops.scan_grid(n, block, items)
    assert grid >= 2  # there is a tile 1 that waits for tile 0
    ws = spmd.ops.workspace(spmd.SCAN_I32, grid, block, n)
    ws.view(torch.int64)[0] = 1  # ticket: epoch 0, next draw 1
    y = torch.zeros_like(x)
    spmd.ops.scan_i32(x, block, items, y=y, ws=ws, stream=stream)
    return y, ws


def test_sync_timeout_then_sync(spmd):
    """A bound of 0 ms while GEMMs of about 10 ms each are still running:
    SPMD_ERR_TIMEOUT, and the work goes on; the next sync waits for it and
    returns OK, with the results correct."""
    import torch

    say("sync timeout")
    n = 8192
    A = torch.from_numpy(synth.normal_f32(synth.SEED_GEMM, n * n).reshape(n, n)).cuda()
    B = torch.from_numpy(synth.normal_f32(synth.SEED_GEMM + 1, n * n).reshape(n, n)).cuda()
    C = torch.empty_like(A)
    spmd.sync()
    for _ in range(3):
        spmd.ops.gemm_f32(A, B, C, 128)
    with pytest.raises(spmd.SpmdError) as e:
        spmd.sync_timeout(ms=0)
    assert e.value.kind == "TIMEOUT"
    spmd.sync()  # waits for the GEMMs; no device error
    spmd.sync_timeout(ms=10000)  # an idle stream: OK at once
    rng = np.random.default_rng(1)
    ii = rng.integers(0, n, 256).astype(np.uint32)
    jj = rng.integers(0, n, 256).astype(np.uint32)
    c64 = oracle.gemm_f64_entries(A.cpu().numpy(), B.cpu().numpy(), ii, jj)
    got = C.cpu().numpy()[ii, jj].astype(np.float64)
    assert np.abs(got - c64).max() / np.abs(c64).max() <= 1e-5 * np.sqrt(n)


def test_device_error_reported_and_cleared(spmd):
    """A look-back that gives up sets the error word: the next sync raises
    SPMD_ERR_DEVICE once and clears it; with the limit restored and a fresh
    workspace the same scan is exact again."""
    import torch

    say("device error: scan ticket skips tile 0, spin limit 256")
    n = 100_003
    x_h = synth.uniform_int32(0xE1, n, 0, 100)
    x = torch.from_numpy(x_h).cuda()
    spmd.sync()
    spmd.set_spin_limit(256)
    try:
        y, _ = _scan_skipping_tile0(spmd, x, 256, 4)
        with pytest.raises(spmd.SpmdError) as e:
            spmd.sync()
        assert e.value.kind == "DEVICE"
    finally:
        spmd.set_spin_limit(0)
    spmd.sync()  # cleared: reported once
    assert np.all(y.cpu().numpy()[:1024] == 0)  # tile 0 (256 x 4 elements) was never scanned
    y = spmd.ops.scan_i32(x, 256, 4)
    spmd.sync()
    assert np.array_equal(y.cpu().numpy(), oracle.scan_i32(x_h, 256, 4))


def test_error_word_is_per_device(spmd):
    """The error word belongs to the device, not to a stream: an error
    raised by a kernel on a side stream is reported by a sync on the main
    stream (and cleared there), after which a sync of the side stream
    reports nothing."""
    import torch

    say("error word shared by streams")
    n = 50_000
    x = torch.from_numpy(synth.uniform_int32(0xE2, n, 0, 100)).cuda()
    side = torch.cuda.Stream()
    spmd.sync()
    side.wait_stream(torch.cuda.current_stream())
    spmd.set_spin_limit(256)
    try:
        _scan_skipping_tile0(spmd, x, 128, 4, stream=side)
        side.synchronize()
    finally:
        spmd.set_spin_limit(0)
    with pytest.raises(spmd.SpmdError) as e:
        spmd.sync()  # the main stream
    assert e.value.kind == "DEVICE"
    spmd.sync(side)
    spmd.sync()


def test_concurrent_persistent_launches(spmd):
    """Three launches whose blocks wait on each other, each sized to fill
    every compute unit, enqueued on three streams at once so that they
    share the device: a scan (512 x 128), a compaction (1024 x 32) and a
    reduction.  Tiles are handed out by each launch's own ticket, so a
    block waits only for tiles that running blocks of its launch hold, and
    every launch completes whatever share of the device the others leave it
    (the queue's forward-progress argument, Section IV).  Five rounds on
    the same workspaces; every result checked."""
    import torch

    n = 1 << 24
    xs = synth.uniform_int32(synth.SEED_SCAN, n, 0, 100)
    xc = synth.uniform_int32(0xC0 + n, n, -1000, 1000)
    xr = synth.uniform_int32(synth.SEED_REDUCE, n, -1000, 1000)
    want_c = oracle.compact_i32(xc, 0)
    want_r = int(xr.astype(np.int64).sum()) % 2**32
    want_s_prefix = oracle.scan_i32(xs[: 1 << 18], 512, 64)
    d_s, d_c, d_r = (torch.from_numpy(a).cuda() for a in (xs, xc, xr))
    ws_s = spmd.ops.workspace(spmd.SCAN_I32, spmd.ops.scan_grid(n, 512, 128), 512, n)
    ws_c = spmd.ops.workspace(spmd.COMPACT_I32, spmd.ops.compact_grid(n, 1024, 32), 1024, n)
    ws_r = spmd.ops.workspace(spmd.REDUCE_I32, 4096, 256, n)
    y_s = torch.empty_like(d_s)
    y_c = torch.empty_like(d_c)
    cnt = torch.empty(1, dtype=torch.int32, device="cuda")
    part = torch.empty(4096, dtype=torch.int32, device="cuda")
    tot = torch.empty(1, dtype=torch.int32, device="cuda")
    streams = [torch.cuda.Stream() for _ in range(3)]
    for rnd in range(5):
        say("concurrent scan + compaction + reduce, round", rnd)
        y_s.fill_(-1)
        cnt.fill_(-1)
        tot.fill_(0)
        torch.cuda.synchronize()
        spmd.ops.scan_i32(d_s, 512, 128, y=y_s, ws=ws_s, stream=streams[0])
        spmd.ops.compact_i32(d_c, 0, 1024, 32, y=y_c, count=cnt, ws=ws_c, stream=streams[1])
        spmd.ops.reduce_i32(d_r, 4096, 256, part, tot, ws_r, stream=streams[2])
        for s in streams:
            s.synchronize()
        spmd.sync()
        assert int(y_s[0].item()) == int(d_s[0].item()), rnd
        assert torch.equal(y_s[1:] - y_s[:-1], d_s[1:]), rnd
        assert np.array_equal(y_s[: 1 << 18].cpu().numpy(), want_s_prefix), rnd
        m = int(cnt.item())
        assert m == want_c.size, (rnd, m)
        assert np.array_equal(y_c[:m].cpu().numpy(), want_c), rnd
        assert int(tot.item()) % 2**32 == want_r, rnd
