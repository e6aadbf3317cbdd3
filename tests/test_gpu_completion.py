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
