"""spmd_launch_noalloc on the GPU: the launch for callers that cannot
allocate, with the classes' workspace taken from the library's static
per-device scratch, against spmd_launch with a caller workspace.

Each class runs two calls in a row on the scratch, the second with a
smaller input (and a smaller grid), and every output must equal, bit for
bit, what spmd_launch writes for the same launch.  A graph captured around
the no-alloc launches is then replayed, with eager launches of the same
class on the same scratch between the replays, and every replay is checked.
"""

import sys

import numpy as np
import pytest

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


def dev(a):
    import torch

    a = np.ascontiguousarray(a)
    return torch.from_numpy(a.view(np.int32) if a.dtype == np.uint32 else a).cuda()


def host(t):
    return t.cpu().numpy()


def _scan_pair(spmd, x, block, items):
    import torch

    n = x.numel()
    G = spmd.ops.scan_grid(n, block, items)
    y_ref = torch.full_like(x, 3)
    y_na = torch.full_like(x, 5)
    ws = spmd.ops.workspace(spmd.SCAN_I32, G, block, n)
    spmd.launch(spmd.SCAN_I32, G, block, 0, [x, y_ref, n, ws])
    spmd.launch_noalloc(spmd.SCAN_I32, G, block, 0, [x, y_na, n])
    spmd.sync()
    return host(y_ref), host(y_na)


def test_noalloc_scan_two_calls(spmd):
    for n, block, items, seed in (((1 << 22) + 12345, 512, 16, 0xA1), (100_003, 256, 4, 0xA2)):
        say("noalloc scan", n, block, items)
        x = dev(synth.uniform_int32(seed, n, 0, 100))
        ref, got = _scan_pair(spmd, x, block, items)
        assert np.array_equal(got, ref), (n, int(np.argmax(got != ref)))


def test_noalloc_reduce_two_calls(spmd):
    import torch

    for n, grid, block, seed in ((1 << 20, 4096, 256, 0xB1), (50_001, 97, 128, 0xB2)):
        say("noalloc reduce", n, grid, block)
        x = dev(synth.uniform_int32(seed, n, -1000, 1000))
        p_ref = torch.full((grid,), 3, dtype=torch.int32, device="cuda")
        p_na = torch.full((grid,), 5, dtype=torch.int32, device="cuda")
        o_ref = torch.full((1,), 3, dtype=torch.int32, device="cuda")
        o_na = torch.full((1,), 5, dtype=torch.int32, device="cuda")
        ws = spmd.ops.workspace(spmd.REDUCE_I32, grid, block, n)
        spmd.launch(spmd.REDUCE_I32, grid, block, 4 * block, [x, p_ref, o_ref, n, ws])
        spmd.launch_noalloc(spmd.REDUCE_I32, grid, block, 4 * block, [x, p_na, o_na, n])
        spmd.sync()
        assert np.array_equal(host(p_na), host(p_ref)), n
        assert int(host(o_na)[0]) == int(host(o_ref)[0]), n


def test_noalloc_compact_two_calls(spmd):
    import torch

    for n, block, items, seed in (((1 << 22) + 7, 1024, 32, 0xC1), (77_777, 256, 8, 0xC2)):
        say("noalloc compact", n, block, items)
        x = dev(synth.uniform_int32(seed, n, -1000, 1000))
        G = spmd.ops.compact_grid(n, block, items)
        y_ref = torch.full_like(x, 3)
        y_na = torch.full_like(x, 3)
        c_ref = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        c_na = torch.full((1,), -2, dtype=torch.int32, device="cuda")
        ws = spmd.ops.workspace(spmd.COMPACT_I32, G, block, n)
        spmd.launch(spmd.COMPACT_I32, G, block, 0, [x, y_ref, c_ref, n, 0, ws])
        spmd.launch_noalloc(spmd.COMPACT_I32, G, block, 0, [x, y_na, c_na, n, 0])
        spmd.sync()
        assert int(host(c_na)[0]) == int(host(c_ref)[0]), n
        assert np.array_equal(host(y_na), host(y_ref)), n


def test_noalloc_graph_replays(spmd):
    """Captured no-alloc scans (two sizes, one after the other) replayed
    three times, with an eager no-alloc scan of another size on the same
    scratch between replays: every replay and every eager launch is exact."""
    import torch

    say("noalloc graph replays")
    xa = dev(synth.uniform_int32(0xD1, 300_001, 0, 100))
    xb = dev(synth.uniform_int32(0xD2, 40_000, 0, 100))
    xc = dev(synth.uniform_int32(0xD3, 123_457, 0, 100))
    want = {}
    for name, x, b, i in (("a", xa, 256, 8), ("b", xb, 128, 4), ("c", xc, 512, 4)):
        ref, _ = _scan_pair(spmd, x, b, i)
        want[name] = ref
    ya, yb, yc = torch.empty_like(xa), torch.empty_like(xb), torch.empty_like(xc)
    Ga, Gb, Gc = (spmd.ops.scan_grid(xa.numel(), 256, 8), spmd.ops.scan_grid(xb.numel(), 128, 4),
                  spmd.ops.scan_grid(xc.numel(), 512, 4))
    spmd.sync()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            spmd.launch_noalloc(spmd.SCAN_I32, Ga, 256, 0, [xa, ya, xa.numel()])
            spmd.launch_noalloc(spmd.SCAN_I32, Gb, 128, 0, [xb, yb, xb.numel()])
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        ya.fill_(-1)
        yb.fill_(-1)
        g.replay()
        spmd.sync()
        assert np.array_equal(host(ya), want["a"]), rep
        assert np.array_equal(host(yb), want["b"]), rep
        yc.fill_(-1)
        spmd.launch_noalloc(spmd.SCAN_I32, Gc, 512, 0, [xc, yc, xc.numel()])
        spmd.sync()
        assert np.array_equal(host(yc), want["c"]), rep


def test_noalloc_rejects_grid_over_region(spmd):
    import torch

    x = torch.zeros(16, dtype=torch.int32, device="cuda")
    y = torch.zeros(16, dtype=torch.int32, device="cuda")
    big = 140_000  # blocks: the workspace exceeds SPMD_NOALLOC_REGION_BYTES
    assert spmd.workspace_size(spmd.SCAN_I32, big, 64, 16) > spmd.NOALLOC_REGION_BYTES
    for kid, args in ((spmd.SCAN_I32, [x, y, 16]), (spmd.REDUCE_I32, [x, y, y, 16]),
                      (spmd.COMPACT_I32, [x, y, y, 16, 0])):
        with pytest.raises(spmd.SpmdError) as e:
            spmd.launch_noalloc(kid, big, 64, 256, args)
        assert e.value.kind == "WORKSPACE"
    spmd.sync()
