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
        items = int(rng.choice([1, 2, 4, 8] if kind == "jacobi" else [1, 2, 4, 8, 16]))
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
