"""The persistent block queue (spmd_batch.h) and the device-side input
generator, on the GPU, against the oracle.

A batch's result must equal each instance run alone by the oracle (bit for
bit: the integer classes are exact and a Jacobi sweep fixes every cell's
rounding), whatever the schedule; eager runs, graph replays and the
one-launch-per-instance baseline must all agree.
"""

import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

KINDS = ("reduce", "scan", "hist", "jacobi")


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


def make_instances(spmd, count, seed, nmax_log2=16, include_edges=True):
    """Mixed instances with host inputs, device buffers and random schedules."""
    import torch

    rng = np.random.default_rng(seed)
    inst = []
    for i in range(count):
        kind = KINDS[i % 4]
        n = int(round(2 ** rng.uniform(0, nmax_log2)))
        if include_edges and i < 16:
            n = [0, 1, 3, 64, 65, 257, 1000, 4099][i // 2 % 8] if kind != "jacobi" else [1, 2, 3, 5][i % 4]
        bd = int(rng.choice([64, 128, 256, 512]))
        items = int(rng.choice([1, 2, 4, 8] if kind == "jacobi" else [1, 2, 4, 8, 16, 32] if kind == "scan"
                               else [1, 2, 4, 8, 16]))
        bpf = int(rng.choice([1, 2, 3, 8, 32]))
        s = 1000 + 7 * i + seed
        if kind == "reduce":
            x = synth.uniform_int32(s, n, -(2**31), 2**31 - 1)
            tin = dev(x) if n else torch.empty(4, dtype=torch.int32, device="cuda")
            tout = torch.empty(1, dtype=torch.int32, device="cuda")
            inst.append(dict(kind=kind, kid=spmd.REDUCE_I32, n=n, ny=1, x=x, tin=tin, tout=tout))
        elif kind == "scan":
            x = synth.uniform_int32(s, n, -(2**31), 2**31 - 1)
            tin = dev(x) if n else torch.empty(4, dtype=torch.int32, device="cuda")
            tout = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
            inst.append(dict(kind=kind, kid=spmd.SCAN_I32, n=n, ny=1, x=x, tin=tin, tout=tout))
        elif kind == "hist":
            x = synth.zipf_u32(s, n) ^ (synth.uniform_u32(s + 1, n) & np.uint32(0xFFFFFF00)) if n else np.zeros(0, np.uint32)
            tin = dev(x) if n else torch.empty(4, dtype=torch.int32, device="cuda")
            tout = torch.full((256,), 77, dtype=torch.int32, device="cuda")
            inst.append(dict(kind=kind, kid=spmd.HIST256_U32, n=n, ny=1, x=x, tin=tin, tout=tout))
        else:
            side = max(1, int(round(np.sqrt(max(n, 1)))))
            ny, nx = side, side + (i % 3)
            x = synth.uniform_f32(s, nx * ny).reshape(ny, nx)
            tin = dev(x)
            tout = torch.empty_like(tin)
            inst.append(dict(kind=kind, kid=spmd.JACOBI5_F32, n=nx, ny=ny, x=x, tin=tin, tout=tout))
        inst[-1].update(bd=bd, sched=(bd, items, bpf))
    return inst


def expected(inst):
    k = inst["kind"]
    x = inst["x"]
    if k == "reduce":
        return np.array([oracle.reduce_i32(x, 1, 64)[1] if x.size else 0], np.int32)
    if k == "scan":
        return oracle.scan_i32(x, 64, 4) if x.size else np.zeros(0, np.int32)
    if k == "hist":
        return oracle.hist256_u32(x, 1, 64).view(np.int32)
    return oracle.jacobi5_f32(x, 16, 16)


def got(inst):
    t = inst["tout"].cpu().numpy()
    if inst["kind"] == "scan":
        return t[: inst["n"]]
    return t


def check_all(insts, what):
    for i, it in enumerate(insts):
        e = expected(it)
        g = got(it)
        assert np.array_equal(g, e), f"{what}: instance {i} {it['kind']} n={it['n']} sched={it['sched']}"


def items_of(insts):
    return [(it["kid"], it["n"], it["ny"], it["bd"], it["tin"], it["tout"]) for it in insts]


def scribble(insts):
    for it in insts:
        it["tout"].fill_(-12345)


@pytest.mark.parametrize("seed", [1, 2])
def test_batch_matches_oracle_all_modes(spmd, seed):
    say("batch mixed 240 instances, seed", seed)
    insts = make_instances(spmd, 240, seed)
    b = spmd.batch.Batch(items_of(insts), [it["sched"] for it in insts])
    st = b.stats()
    assert st["persistent_launches"] >= 2 and st["blocks"] > 0
    say("eager persistent")
    scribble(insts)
    b.launch()
    spmd.sync()
    check_all(insts, "persistent")
    for rep in range(3):
        say("graph replay", rep)
        scribble(insts)
        b.graph_launch()
        spmd.sync()
        check_all(insts, f"graph replay {rep}")
    say("one launch per instance")
    scribble(insts)
    b.launch_each()
    spmd.sync()
    check_all(insts, "launch_each")
    b.close()


def test_batch_single_large_instances(spmd):
    """A few large instances: many chunks per instance, scan tiles fetched
    across many workers, reduce last-block protocol over thousands of
    blocks."""
    import torch

    say("batch large instances")
    insts = []
    n = 3_000_001
    x = synth.uniform_int32(5, n, -(2**31), 2**31 - 1)
    for kid, kind, sched in [(spmd.REDUCE_I32, "reduce", (256, 1, 1)), (spmd.SCAN_I32, "scan", (512, 4, 2)),
                             (spmd.SCAN_I32, "scan", (64, 1, 1))]:
        tout = torch.empty(n if kind == "scan" else 1, dtype=torch.int32, device="cuda")
        insts.append(dict(kind=kind, kid=kid, n=n, ny=1, x=x, tin=dev(x), tout=tout, bd=sched[0], sched=sched))
    u = synth.uniform_f32(6, 1500 * 1700).reshape(1500, 1700)
    insts.append(dict(kind="jacobi", kid=spmd.JACOBI5_F32, n=1700, ny=1500, x=u, tin=dev(u),
                      tout=torch.empty((1500, 1700), dtype=torch.float32, device="cuda"), bd=512, sched=(512, 8, 4)))
    b = spmd.batch.Batch(items_of(insts), [it["sched"] for it in insts])
    for rep in range(2):
        scribble(insts)
        b.graph_launch()
        spmd.sync()
        check_all(insts, f"large rep {rep}")
    b.close()


def test_batch_few_workers(spmd):
    """One worker per CU and group: the queue must still drain, and scan
    look-back must still progress with few resident tiles."""
    say("batch 1 worker per CU")
    insts = make_instances(spmd, 64, 9, nmax_log2=18, include_edges=False)
    b = spmd.batch.Batch(items_of(insts), [it["sched"] for it in insts], workers_per_cu=1)
    scribble(insts)
    b.launch()
    spmd.sync()
    check_all(insts, "1 worker/CU")
    b.close()


@pytest.mark.parametrize("start,count", [(0, 1000), (123456789, 4099)])
def test_device_generator_matches_host(spmd, start, count):
    import torch

    say("device generator", start, count)
    t = torch.empty(count, dtype=torch.int32, device="cuda")
    spmd.batch.synth_uniform_i32(t, synth.SEED_SCAN, -1000, 1000, start)
    assert np.array_equal(t.cpu().numpy(), synth.uniform_int32(synth.SEED_SCAN, count, -1000, 1000, start))
    spmd.batch.synth_uniform_i32(t, 7, -(2**31), 2**31 - 1, start)
    assert np.array_equal(t.cpu().numpy(), synth.uniform_int32(7, count, -(2**31), 2**31 - 1, start))
    f = torch.empty(count, dtype=torch.float32, device="cuda")
    spmd.batch.synth_uniform_f32(f, synth.SEED_JACOBI, start)
    assert np.array_equal(f.cpu().numpy(), synth.uniform_f32(synth.SEED_JACOBI, count, start))
    spmd.batch.synth_raw_u32(t, 3, start)
    assert np.array_equal(t.cpu().numpy().view(np.uint32), synth.uniform_u32(3, count, start))
    cdf = torch.from_numpy(synth.zipf_cdf(1.1, 256)).cuda()
    spmd.batch.synth_zipf_u32(t, synth.SEED_HIST, cdf, start)
    assert np.array_equal(t.cpu().numpy().view(np.uint32), synth.zipf_u32(synth.SEED_HIST, count, start=start))
    spmd.sync()


def test_mixed_workload_small(spmd):
    """The mixed-launch workload generator end to end at small sizes: device
    inputs equal the host generator's, batch outputs equal the oracle's."""
    from paper_2206_07896_amd import workload as W

    say("mixed workload 200 instances, n in [2^4, 2^14]")
    specs = W.mixed_specs(200, seed=0xC4, log2_lo=4, log2_hi=14)
    data = W.MixedData(specs)
    sched = W.as_launched_schedules(specs)
    b = spmd.batch.Batch(data.items(), sched)
    b.graph_launch()
    spmd.sync()
    for i, s in enumerate(specs):
        x = data.host_input(i)
        assert np.array_equal(data.input_of(i).cpu().numpy().reshape(x.shape).view(x.dtype), x), i
        got = data.output_of(i).cpu().numpy()
        k = W.KIND_NAMES[s["kid"]]
        if k == "reduce":
            assert int(got[0]) == int(x.astype(np.int64).sum()), i
        elif k == "scan":
            assert np.array_equal(got, oracle.scan_i32(x, 64, 4)), i
        elif k == "hist":
            assert np.array_equal(got.view(np.uint32), oracle.hist256_u32(x, 1, 64)), i
        else:
            assert np.array_equal(got, oracle.jacobi5_f32(x, 16, 16)), i
    b.close()


def test_batch_hist_skew(spmd):
    """Skewed and one-bin histogram instances through the queue's fused
    chunk body under several schedules."""
    import torch

    perm = synth.bin_permutation()
    insts = []
    for i, (alpha, n, sched) in enumerate([(0.0, 100003, (256, 4, 8)), (2.0, 1 << 18, (512, 16, 1)),
                                           (3.0, 262147, (64, 1, 32)), ("one", 50000, (128, 8, 3)),
                                           (2.0, 1 << 18, (1024 // 4, 16, 32)), (3.0, 4099, (512, 2, 2))]):
        upper = synth.uniform_u32(70 + i, n) & np.uint32(0xFFFFFF00)
        if alpha == "one":
            x = upper | np.uint32(200)
        else:
            x = synth.permute_bins(synth.zipf_u32(60 + i, n, alpha) | upper, perm) if i % 2 else \
                synth.zipf_u32(60 + i, n, alpha) | upper
        insts.append(dict(kind="hist", kid=spmd.HIST256_U32, n=n, ny=1, x=x, tin=dev(x),
                          tout=torch.full((256,), 77, dtype=torch.int32, device="cuda"), bd=256, sched=sched))
    say("batch hist skew", [it["sched"] for it in insts])
    b = spmd.batch.Batch(items_of(insts), [it["sched"] for it in insts])
    for mode in ("eager", "graph", "graph"):
        scribble(insts)
        b.launch() if mode == "eager" else b.graph_launch()
        spmd.sync()
        check_all(insts, f"hist skew {mode}")
    b.close()


@pytest.mark.parametrize("wpc", [0, 1])
def test_batch_chunk_ranges(spmd, wpc):
    """A segment's chunks are cut into up to 8 ranges, one cursor each, with
    static first chunks and stealing across ranges.  One histogram instance
    per batch, blockDim 64, 1 item, 1 block per fetch, so chunks = blocks:
    counts around the range count (1, 3, 7, 8, 9) and around the worker pool
    (all static, one dynamic chunk, several per worker), ragged last blocks."""
    import torch

    pool = spmd.batch.pool_size(spmd.HIST256_U32, 64, wpc)
    counts = [1, 3, 7, 8, 9, pool - 1, pool, pool + 1, 3 * pool + 5]
    for j, chunks in enumerate(counts):
        n = 64 * (chunks - 1) + 17
        x = synth.uniform_u32(90 + j, n)
        inst = dict(kind="hist", kid=spmd.HIST256_U32, n=n, ny=1, x=x, tin=dev(x),
                    tout=torch.full((256,), 77, dtype=torch.int32, device="cuda"), bd=64, sched=(64, 1, 1))
        say("chunk ranges", wpc, chunks, "of pool", pool)
        b = spmd.batch.Batch(items_of([inst]), [inst["sched"]], workers_per_cu=wpc)
        assert b.stats()["chunks"] == chunks
        for mode in ("eager", "graph", "graph"):
            scribble([inst])
            b.launch() if mode == "eager" else b.graph_launch()
            spmd.sync()
            check_all([inst], f"chunk ranges {chunks} {mode}")
        b.close()


@pytest.mark.parametrize("wpc", [0, 1])
def test_batch_scan_ranges(spmd, wpc):
    """Scan segments of small tiles are cut into chunk ranges at instance
    starts, every tile drawn from its range's cursor in order.  Many
    instances of ragged sizes plus one long instance (hundreds of tiles, so
    look-backs run deep inside a range and a range boundary falls right
    after it), at 64- and 256-element tiles; with one worker per CU the
    ranges are drained by few workers and stolen from."""
    import torch

    rng = np.random.default_rng(31 + wpc)
    sizes = [int(v) for v in rng.integers(1, 3000, 60)]
    sizes[17] = 200_003
    insts = []
    for j, n in enumerate(sizes):
        x = synth.uniform_int32(400 + j, n, 0, 100)
        sched = (64, 1, 1) if j % 2 else (128, 2, 1)
        insts.append(dict(kind="scan", kid=spmd.SCAN_I32, n=n, ny=1, x=x, tin=dev(x),
                          tout=torch.zeros(n + 64, dtype=torch.int32, device="cuda"), bd=256, sched=sched))
    say("scan ranges", wpc, len(insts), "instances")
    b = spmd.batch.Batch(items_of(insts), [it["sched"] for it in insts], workers_per_cu=wpc)
    for mode in ("eager", "graph", "graph"):
        scribble(insts)
        b.launch() if mode == "eager" else b.graph_launch()
        spmd.sync()
        check_all(insts, f"scan ranges {mode}")
        for it in insts:  # nothing written past the end
            assert (host(it["tout"])[it["n"]:] == -12345).all(), f"scan ranges {mode}: n={it['n']}"
    b.close()


def test_batch_wide_scan(spmd):
    """Scans of 32 items per thread run in a queue class of their own, side
    by side with ordinary scan tiles in the same level: ragged and aligned
    sizes, a misaligned view (the item path), all four block sizes."""
    import torch

    cases = [(1, (64, 32, 1)), (2047, (64, 32, 4)), (2048, (64, 32, 1)), (100_003, (128, 32, 1)),
             (1 << 20, (256, 32, 2)), ((1 << 20) + 3, (512, 32, 1)), (300_001, (512, 16, 1)),
             (65_537, (256, 8, 1)), (50_000, (512, 32, 1))]
    insts = []
    for j, (n, sched) in enumerate(cases):
        x = synth.uniform_int32(500 + j, n, -(2**31), 2**31 - 1)
        if j == 8:  # input one element into its buffer: not 16-byte aligned
            buf = dev(np.concatenate([np.zeros(1, np.int32), x]))
            tin = buf[1:]
        else:
            tin = dev(x)
        insts.append(dict(kind="scan", kid=spmd.SCAN_I32, n=n, ny=1, x=x, tin=tin,
                          tout=torch.zeros(n + 64, dtype=torch.int32, device="cuda"), bd=256, sched=sched))
    say("wide scan", [it["sched"] for it in insts])
    b = spmd.batch.Batch(items_of(insts), [it["sched"] for it in insts])
    for mode in ("eager", "graph", "graph"):
        scribble(insts)
        b.launch() if mode == "eager" else b.graph_launch()
        spmd.sync()
        check_all(insts, f"wide scan {mode}")
        for it in insts:
            assert (host(it["tout"])[it["n"]:] == -12345).all(), f"wide scan {mode}: n={it['n']}"
    b.launch_each()
    spmd.sync()
    check_all(insts, "wide scan, one launch per instance")
    b.close()


@pytest.mark.parametrize("seed", [5])
def test_batch_random_levels(spmd, seed):
    """Seeded instances with random dependencies (no data flows along them):
    many levels, several queues per level, every output still the
    oracle's."""
    rng = np.random.default_rng(seed)
    insts = make_instances(spmd, 48, seed, nmax_log2=14)
    deps = [None if i == 0 or rng.random() < 0.4 else int(rng.integers(0, i)) for i in range(len(insts))]
    for it in insts:  # about one in five runs as its own grid (bpf 0)
        if rng.random() < 0.2:
            it["sched"] = (it["sched"][0], it["sched"][1], 0)
    say("random levels", seed, deps, [it["sched"] for it in insts])
    b = spmd.batch.Batch(items_of(insts), [it["sched"] for it in insts], deps=deps)
    for mode in ("eager", "graph", "graph"):
        scribble(insts)
        b.launch() if mode == "eager" else b.graph_launch()
        spmd.sync()
        check_all(insts, f"random levels {mode}")
    b.close()


# --------------------------------------------------------------------------
# Dependent instances (spmd_batch_create_dep)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("nx", [517, 516])
@pytest.mark.parametrize("sched", [(256, 4, 8), (64, 1, 3), (512, 8, 32), (256, 4, 0), (128, 2, 0)])
def test_dependent_jacobi_chain_in_one_batch(spmd, sched, nx):
    """25 sweeps as 25 instances of one batch, each reading the previous
    one's output (nx 516 also takes the 16-byte body when a sweep runs as its
    own grid), bit-exact against 25 sweeps of the oracle, eagerly and over
    graph replays."""
    import torch

    ny, sweeps = 131, 25
    say("dependent jacobi chain", ny, nx, sweeps, sched)
    u = synth.uniform_f32(0xD5, ny * nx).reshape(ny, nx)
    bufs = [dev(u), torch.empty((ny, nx), dtype=torch.float32, device="cuda")]
    items = [(spmd.JACOBI5_F32, nx, ny, 256, bufs[t % 2], bufs[(t + 1) % 2]) for t in range(sweeps)]
    deps = [None] + list(range(sweeps - 1))
    b = spmd.batch.Batch(items, [sched] * sweeps, deps=deps)
    want = oracle.jacobi5_f32_sweeps(u, sweeps)
    for mode in ("eager", "graph", "graph"):
        bufs[0].copy_(torch.from_numpy(u))
        bufs[1].fill_(-1.0)
        b.launch() if mode == "eager" else b.graph_launch()
        spmd.sync()
        assert np.array_equal(host(bufs[sweeps % 2]), want), mode
    b.close()


def test_dependency_across_queues(spmd):
    """Three levels over queues in both orders: a Jacobi sweep, a scan of
    its output bits (the SCAN queue comes before the JACOBI queue in the
    group order), a histogram of the scan, and an independent reduction
    beside them at level 0."""
    import torch

    say("jacobi -> scan -> hist dependency, reduce beside")
    ny, nx = 300, 517
    n = ny * nx
    u = synth.uniform_f32(0xD6, n).reshape(ny, nx)
    ut = dev(u)
    v = torch.empty_like(ut)
    y = torch.empty((n,), dtype=torch.int32, device="cuda")
    h = torch.full((256,), 5, dtype=torch.int32, device="cuda")
    r_in = synth.uniform_int32(0xD7, 70001, -1000, 1000)
    r_x = dev(r_in)
    r = torch.zeros((1,), dtype=torch.int32, device="cuda")
    items = [(spmd.JACOBI5_F32, nx, ny, 256, ut, v), (spmd.SCAN_I32, n, 1, 256, v.view(torch.int32), y),
             (spmd.HIST256_U32, n, 1, 256, y, h), (spmd.REDUCE_I32, r_in.size, 1, 256, r_x, r)]
    sched = [(256, 2, 4), (256, 8, 1), (256, 16, 4), (256, 4, 2)]
    b = spmd.batch.Batch(items, sched, deps=[None, 0, 1, None])
    want_v = oracle.jacobi5_f32(u, 16, 16)
    want_y = oracle.scan_i32(want_v.view(np.int32).ravel(), 64, 4)
    want_h = oracle.hist256_u32(want_y.view(np.uint32), 1, 64)
    want_r = int(oracle.reduce_i32(r_in, 1, 64)[1])
    for mode in ("eager", "graph", "graph"):
        v.fill_(-1.0)
        y.fill_(0)
        r.fill_(7)
        b.launch() if mode == "eager" else b.graph_launch()
        spmd.sync()
        assert np.array_equal(host(v), want_v), mode
        assert np.array_equal(host(y), want_y), mode
        assert np.array_equal(host(h).view(np.uint32), want_h), mode
        assert int(host(r)[0]) == want_r, mode
    b.close()


def _launch_desc(spmd, W, data, i):
    """Instance i of a mixed workload as the CUDA launch it stands for: its
    blockDim, 4 elements per thread (JACOBI: 64-wide blocks, 4 cells down a
    column), the packed arguments of spmd_launch."""
    s = data.specs[i]
    k, bd = s["kid"], s["block_dim"]
    x, y = data.input_of(i), data.output_of(i)
    if k == spmd.JACOBI5_F32:
        by = bd // 64
        grid = (-(-s["nx"] // 64), -(-s["ny"] // (by * 4)))
        return (k, grid, (64, by), 0, [x, y, s["nx"], s["ny"]])
    grid = (max(1, -(-s["n"] // (bd * 4))),)
    if k == spmd.REDUCE_I32:
        return (k, grid, (bd,), 4 * bd, [x, y, y, s["n"], y])  # the batch writes `out` only
    if k == spmd.SCAN_I32:
        return (k, grid, (bd,), 0, [x, y, s["n"], y])           # workspace unused in a batch
    return (k, grid, (bd,), 0, [x, y, s["n"]])


def _oracle_of(W, data, i):
    s = data.specs[i]
    x = data.host_input(i)
    k = W.KIND_NAMES[s["kid"]]
    if k == "reduce":
        return np.array([oracle.reduce_i32(x, 1, 64)[1]], np.int32)
    if k == "scan":
        return oracle.scan_i32(x, 64, 4)
    if k == "hist":
        return oracle.hist256_u32(x, 1, 64).view(np.int32)
    return oracle.jacobi5_f32(x, 16, 16)


@pytest.mark.timeout(900)
def test_mixed_workload_configured_size(spmd):
    """The measured mixed workload at its configured size: 10 000 launches,
    class uniform over the four batchable classes, n = round(2^U) with
    U ~ U[10, 22] (about 5e9 elements), blockDim uniform over 64..512, run
    by spmd_launch_batch under SPMD_SCHED_LEARNED with the shipped cost
    model, its fallback threshold (low-confidence launches are tuned
    exhaustively first) and its batch slack.  Every instance with n <= 2^14 and a seeded sample
    of 200 larger ones are compared with the oracle; the whole output arena
    must then equal, byte for byte, the batch-aware learned plan that the
    measurement replays from a graph (model choice without fallback) and
    the one-launch-per-instance baseline."""
    import torch

    from paper_2206_07896_amd import learned as L
    from paper_2206_07896_amd import workload as W

    model = L.load_default()
    assert model is not None, "the package ships a cost model"
    specs = W.mixed_specs(10000)
    data = W.MixedData(specs)
    launches = [_launch_desc(spmd, W, data, i) for i in range(len(specs))]
    say("mixed workload 10000 launches, SCHED_LEARNED, tau", model.tau)
    model.load()
    try:
        data.outputs.fill_(-1)
        ws = spmd.batch.launch_batch(launches, spmd.batch.SCHED_LEARNED)
        spmd.sync()
        rep = spmd.batch.launch_batch_report()
        del ws
    finally:
        spmd.batch.model_load(model.params[:0], model.norm, 0.0)  # unload
    say("report", rep)
    assert rep["launches"] == 10000 and rep["by_model"] + rep["tuned"] + rep["cached"] == 10000
    assert rep["by_model"] > 0
    got_all = data.outputs.clone()
    small = [i for i, s in enumerate(specs) if s["n"] <= 1 << 14]
    large = [i for i, s in enumerate(specs) if s["n"] > 1 << 14]
    rng = np.random.default_rng(0xC4)
    sample = sorted(rng.choice(large, 200, replace=False).tolist())
    say("oracle checks", len(small), "small +", len(sample), "large")
    assert len(small) > 2500
    for i in small + sample:
        want = _oracle_of(W, data, i)
        g = data.output_of(i).cpu().numpy()
        assert np.array_equal(g, want.reshape(g.shape)), (i, specs[i]["kid"], specs[i]["n"])
    # the measured plan (batch-aware learned choice, graph replay) and the baseline
    choice, _, _ = model.choose(specs, slack=model.slack)
    b = spmd.batch.Batch(data.items(), [L.CANDIDATES[j] for j in choice])
    for mode in ("graph", "graph", "each"):
        say("mixed workload 10000", mode)
        data.outputs.fill_(-1)
        b.graph_launch() if mode == "graph" else b.launch_each()
        spmd.sync()
        assert bool(torch.equal(data.outputs, got_all)), mode
    b.close()
    del data
    torch.cuda.empty_cache()


def test_hist_bins_cleared_at_their_own_level(spmd):
    """One 256-bin buffer read and rewritten across dependency levels: scan
    of its prior contents (level 0), histogram of keys A into it (1), scan
    of those counts (2), histogram of keys B into it (3).  Each histogram
    overwrites the bins at its own level, so the first scan sees the prior
    contents and the buffer ends as the counts of B alone."""
    import torch

    say("hist bins across levels")
    prior = synth.uniform_int32(0xB1, 256, -1000, 1000)
    ka = synth.zipf_u32(0xB2, 50001)
    kb = synth.zipf_u32(0xB3, 70003) ^ (synth.uniform_u32(0xB4, 70003) & np.uint32(0xFFFFFF00))
    h = dev(prior)
    s1 = torch.empty(256, dtype=torch.int32, device="cuda")
    s2 = torch.empty(256, dtype=torch.int32, device="cuda")
    ta, tb = dev(ka), dev(kb)
    items = [(spmd.SCAN_I32, 256, 1, 64, h, s1), (spmd.HIST256_U32, ka.size, 1, 256, ta, h),
             (spmd.SCAN_I32, 256, 1, 128, h, s2), (spmd.HIST256_U32, kb.size, 1, 512, tb, h)]
    cnt_a = oracle.hist256_u32(ka, 1, 64)
    want_s1 = oracle.scan_i32(prior, 64, 4)
    want_s2 = oracle.scan_i32(cnt_a.view(np.int32), 64, 4)
    want_h = oracle.hist256_u32(kb, 1, 64)
    for scheds in ([(64, 1, 1), (256, 4, 2), (128, 2, 1), (512, 8, 1)],     # every level through the queue
                   [(64, 1, 1), (256, 4, 0), (128, 2, 1), (512, 8, 0)]):    # histograms as their own grids
        b = spmd.batch.Batch(items, scheds, deps=[None, 0, 1, 2])
        for mode in ("eager", "graph", "graph"):
            h.copy_(torch.from_numpy(prior).cuda())
            s1.fill_(0)
            s2.fill_(0)
            b.launch() if mode == "eager" else b.graph_launch()
            spmd.sync()
            assert np.array_equal(host(s1), want_s1), (scheds, mode)
            assert np.array_equal(host(s2), want_s2), (scheds, mode)
            assert np.array_equal(host(h).view(np.uint32), want_h), (scheds, mode)
        b.close()


def test_output_over_input_rejected(spmd):
    """An in-place scan or compaction, and a batch instance whose output
    overlaps its input, are refused before any work is enqueued (a batch may
    run an instance several times: graph replays, the fallback's timing)."""
    import torch

    say("overlap rejected")
    x = torch.arange(1000, dtype=torch.int32, device="cuda")
    keep = x.clone()
    ws = spmd.ops.workspace(spmd.SCAN_I32, 16, 64, 1000)
    for y in (x, x[10:]):  # in place, and shifted by 10 elements
        with pytest.raises(spmd.SpmdError) as e:
            spmd.launch(spmd.SCAN_I32, 16, 64, 0, [x[: y.numel()], y, y.numel(), ws])
        assert e.value.kind == "ARGS"
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(spmd.SpmdError) as e:
        spmd.ops.compact_i32(x, 0, y=x, count=cnt)
    assert e.value.kind == "ARGS"
    with pytest.raises(spmd.SpmdError) as e:
        spmd.batch.Batch([(spmd.SCAN_I32, 1000, 1, 256, x, x)], [(256, 4, 1)])
    assert e.value.kind == "ARGS"
    with pytest.raises(spmd.SpmdError) as e:
        spmd.batch.launch_batch([(spmd.SCAN_I32, (4,), (256,), 0, [x, x, 1000, ws])], spmd.batch.SCHED_AS_LAUNCHED)
    assert e.value.kind == "ARGS"
    spmd.sync()
    assert bool(torch.equal(x, keep))
