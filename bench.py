"""Benchmark of the SPMD kernel-grid executor on one MI355X.

One step = one pass of the warp-primitive workload through the C ABI:
  * SCAN_I32 over 2^26 int32 uniform in [0, 100], blockDim 512 (64 items
    per thread, single pass with decoupled look-back), then
  * HIST256_U32 over 2^27 uint32 keys drawn Zipf(1.1) over 256 bins with
    per-block LDS sub-histograms.
Algorithmic bytes per step: 8 B per scanned element (read x, write y) +
4 B per key + the 1 KiB histogram.  Inputs are generated once (seeded),
resident in HBM before timing, and rotated between two copies so that each
step reads data the previous step did not touch (the rotation set is larger
than the 256 MB Infinity Cache).

Printed: one JSON line (metric, value = GB/s of the whole step, roofline of
the dominant kernel measured with HIP events on the launch stream, the CPU
oracle on the same workload, and per-kernel figures of the other
workloads: the block reduction, the Jacobi stencil and the fp32 GEMM).
Progress goes to stderr.
"""

from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, 8 TB/s
FP32_MFMA_PEAK_TFS = 157.3     # MI355X dense fp32 matrix

SCAN_N = 1 << 26
HIST_N = 1 << 27
SCAN_BLOCK, SCAN_ITEMS = 512, 128
HIST_GRID, HIST_BLOCK = 256, 1024
SETTLE_S = 0.5  # untimed repetitions of the step before the warm-up steps


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def to_dev(a):
    import torch

    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).cuda()


class Timer:
    """HIP events recorded on torch's current stream, which is the stream
    every launch of this benchmark goes to."""

    def __init__(self):
        import torch

        self.torch = torch
        self.pairs = []

    def start(self):
        e = self.torch.cuda.Event(enable_timing=True)
        e.record()
        return e

    def stop(self, s):
        e = self.torch.cuda.Event(enable_timing=True)
        e.record()
        self.pairs.append((s, e))

    def mean_ms(self):
        return sum(s.elapsed_time(e) for s, e in self.pairs) / max(1, len(self.pairs))

    def median_ms(self):
        v = sorted(s.elapsed_time(e) for s, e in self.pairs)
        return v[len(v) // 2] if v else 0.0


def measure(fn, reps, warmup=2):
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t = Timer()
    for _ in range(reps):
        s = t.start()
        fn()
        t.stop(s)
    torch.cuda.synchronize()
    return t.median_ms()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip the other workloads")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-launch queue")
    ap.add_argument("--mixed-count", type=int, default=10000)
    ap.add_argument("--learned-eval", type=int, default=0, metavar="HELDOUT",
                    help="also tune, train and score the cost model on this many held-out launches "
                         "(500 training launches; minutes of GPU time)")
    ap.add_argument("--regret-count", type=int, default=200,
                    help="held-out launches timed under every schedule to score the shipped cost model (0: skip)")
    ap.add_argument("--only-step", action="store_true",
                    help="run only the timed step (for profiler runs): no extras, mixed queue or CPU baseline")
    ap.add_argument("--only-gemm", action="store_true",
                    help="run only the fp32 GEMM at tiles 64, 128 and 256, a few launches each (for profiler runs)")
    ap.add_argument("--only", choices=("reduce", "scan", "jacobi", "compact", "chain", "hist", "mixed"), default=None,
                    help="run only one other workload, then three 256 MiB calibration copies (for profiler runs)")
    ap.add_argument("--gemm-n", type=int, default=4096, help="M = N = K of --only-gemm")
    args = ap.parse_args()
    if args.only_step:
        args.no_cpu = args.no_extra = args.no_mixed = True
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (each kernel class "
              "would shard over GPUs with at most one collective exchange)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2206_07896_amd as spmd
    import synth

    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    if args.only_gemm:
        print(json.dumps({"only_gemm": gemm_workloads(spmd, synth, reps=5, n=args.gemm_n)}), flush=True)
        return
    if args.only:
        fn = {"reduce": reduce_workloads, "scan": scan_size_workloads, "jacobi": jacobi_workloads,
              "compact": compact_workloads,
              "chain": chain_workloads, "hist": hist_contention_workloads,
              "mixed": lambda sp, _sy: mixed_queue(sp, args.mixed_count, reps=3)}[args.only]
        out = fn(spmd, synth)
        calibration_copies()
        print(json.dumps({f"only_{args.only}": out}), flush=True)
        return

    log("generating inputs")
    xs_h = synth.uniform_int32(synth.SEED_SCAN, SCAN_N, 0, 100)
    ks_h = synth.zipf_u32(synth.SEED_HIST, HIST_N)
    xs = [to_dev(xs_h), to_dev(xs_h)]
    ks = [to_dev(ks_h), to_dev(ks_h)]
    ys = [torch.empty_like(xs[0]) for _ in range(2)]
    hist = torch.empty(256, dtype=torch.int32, device="cuda")
    scan_grid = spmd.ops.scan_grid(SCAN_N, SCAN_BLOCK, SCAN_ITEMS)
    ws = spmd.ops.workspace(spmd.SCAN_I32, scan_grid, SCAN_BLOCK, SCAN_N)

    # Timed launches carry HIP events bound to their kernel dispatches
    # (spmd_launch_timed), not marker packets.  The scan, the dominant
    # kernel, binds a start and a stop event: its span is its kernel's device
    # time.  The histogram binds only a stop event, which costs the stream
    # nothing (a bound start event costs about a marker); its span runs from
    # the scan's stop, so it also holds the gaps before its two dispatches.
    def step(i, ev=None):
        spmd.ops.scan_i32(xs[i & 1], SCAN_BLOCK, SCAN_ITEMS, y=ys[i & 1], ws=ws, events=ev and (ev[0], ev[1]))
        spmd.ops.hist256_u32(ks[i & 1], HIST_GRID, HIST_BLOCK, hist=hist, events=ev and (None, ev[2]))

    # Settle: repeat the step untimed for half a second first, so the timed
    # steps do not run while the GPU's clocks are still ramping up from idle
    # (on a fresh box the first milliseconds of HBM-bound work run ~8% slow).
    t_settle = time.perf_counter()
    i = 0
    while time.perf_counter() - t_settle < SETTLE_S:
        for _ in range(8):
            step(i)
            i += 1
        torch.cuda.synchronize()
    for i in range(args.warmup):
        step(i)
    spmd.sync()

    evs = [spmd.timing_events(3) for _ in range(args.steps)]
    torch.cuda.synchronize()
    # as timeit does: no cyclic-GC pass of the host harness inside the timed
    # steps (one would leave the GPU idle for milliseconds)
    gc.collect()
    gc.disable()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(args.warmup + i, evs[i])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gc.enable()
    t_scan, t_hist = Timer(), Timer()
    t_scan.pairs = [(e[0], e[1]) for e in evs]
    t_hist.pairs = [(e[1], e[2]) for e in evs]
    spmd.sync()  # raises if a kernel reported a device-side error
    ms_per_step = (t1 - t0) * 1e3 / args.steps

    # spot check of the last step's outputs (full parity lives in the tests)
    last = (args.warmup + args.steps - 1) & 1
    y = ys[last].cpu().numpy().view(np.uint32)
    assert int(y[-1]) == int(xs_h.astype(np.int64).sum()) % 2**32
    h = hist.cpu().numpy().view(np.uint32)
    assert int(h.astype(np.int64).sum()) == HIST_N

    if args.only_step:
        calibration_copies()

    scan_bytes = 8 * SCAN_N
    hist_bytes = 4 * HIST_N + 1024
    step_bytes = scan_bytes + hist_bytes
    value = step_bytes / (ms_per_step * 1e-3) / 1e9
    ms_scan, ms_hist = t_scan.mean_ms(), t_hist.mean_ms()
    scan_gbs = scan_bytes / (ms_scan * 1e-3) / 1e9
    hist_gbs = hist_bytes / (ms_hist * 1e-3) / 1e9
    log(f"step {ms_per_step:.4f} ms  scan {ms_scan * 1e3:.1f} us {scan_gbs:.0f} GB/s  "
        f"hist {ms_hist * 1e3:.1f} us {hist_gbs:.0f} GB/s")
    if ms_scan >= ms_hist:
        dom = (f"scan_i32_kernel<{SCAN_BLOCK},{SCAN_ITEMS}>", scan_bytes, ms_scan, scan_gbs)
    else:
        dom = (f"hist256_kernel<{HIST_BLOCK}>", hist_bytes, ms_hist, hist_gbs)
    roofline = {
        "kernel": dom[0],
        "bound": "hbm",
        "achieved": round(dom[3], 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(dom[3] / HBM_PEAK_GBS, 4),
        "traffic": measured_traffic(dom[0]),
        "bytes_per_launch": dom[1],
        "avg_launch_us": round(dom[2] * 1e3, 2),
        "timing": "HIP events bound to the scan's first and last kernel dispatch (spmd_launch_timed) on the "
                  "launch stream, every timed step; the histogram's span runs from the scan's stop to its own "
                  "bound stop event",
    }

    kernels = {
        f"scan_i32 2^26 b{SCAN_BLOCK} i{SCAN_ITEMS}": {"us": round(ms_scan * 1e3, 2), "GB/s": round(scan_gbs, 1),
                               "frac_hbm": round(scan_gbs / HBM_PEAK_GBS, 4)},
        "hist256_u32 2^27 zipf1.1 g256 b1024": {"us": round(ms_hist * 1e3, 2), "GB/s": round(hist_gbs, 1),
                                                "frac_hbm": round(hist_gbs / HBM_PEAK_GBS, 4)},
    }
    del xs, ks, ys
    torch.cuda.empty_cache()
    if not args.no_extra:
        kernels.update(extra_workloads(spmd, synth))

    mixed = None
    if not args.no_mixed:
        mixed = mixed_queue(spmd, args.mixed_count)

    regret = None
    if args.regret_count and not args.no_mixed:
        from paper_2206_07896_amd import learned as L

        model = L.load_default()
        if model is not None:
            log(f"schedule regret: {args.regret_count} held-out launches x every schedule")
            regret = L.heldout_regret(model, args.regret_count)
            log(f"schedule regret: {json.dumps(regret)}")
        torch.cuda.empty_cache()

    learned_eval = None
    if args.learned_eval:
        from paper_2206_07896_amd import learned as L

        learned_eval, _ = L.evaluate(train_count=500, heldout_count=args.learned_eval, log=log)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(xs_h, ks_h, step_bytes)
        del xs_h, ks_h
        extra_cpu = cpu_executor_baselines(args.mixed_count)
        for key, rec in extra_cpu.items():
            if key == "mixed_queue":
                if mixed is not None:
                    mixed["cpu_oracle"] = rec
            else:
                kernels.setdefault(key, {})["cpu_oracle"] = rec

    out = {
        "metric": "GB/s & % HBM peak per kernel; mixed-queue launches/s, persistent vs 1-by-1",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (seeded SplitMix64: uniform int32 [0,100], Zipf(1.1) keys)",
        "config": {
            "workload": "warp-primitive workload: inclusive scan of 2^26 int32 U[0,100] (blockDim 512) "
                        "+ 256-bin atomic histogram of 2^27 u32 Zipf(1.1) keys (LDS sub-histograms)",
            "scan_n": SCAN_N, "scan_block": SCAN_BLOCK, "scan_items": SCAN_ITEMS,
            "hist_n": HIST_N, "hist_grid": HIST_GRID, "hist_block": HIST_BLOCK,
            "bytes_per_step": step_bytes,
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": kernels,
        "mixed_queue": mixed,
        "schedule_regret": regret,
    }
    if learned_eval is not None:
        out["learned_schedule_eval"] = learned_eval
    print(json.dumps(out), flush=True)


def calibration_copies():
    """Three device copies of 256 MiB: a kernel of known traffic, for scaling
    hardware byte counters in profiler runs."""
    import torch

    src = torch.ones(1 << 26, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def extra_workloads(spmd, synth):
    """Per-kernel figures of the other workloads (not part of the step)."""
    res = copy_reference()
    res.update(vendor_scan_reference(synth))
    res.update(scan_size_workloads(spmd, synth))
    res.update(reduce_workloads(spmd, synth))
    res.update(jacobi_workloads(spmd, synth))
    res.update(hist_contention_workloads(spmd, synth))
    res.update(compact_workloads(spmd, synth))
    res.update(chain_workloads(spmd, synth))
    res.update(gemm_workloads(spmd, synth))
    return res


def copy_reference():
    """A plain device copy of 256 MiB (read + write): reference, and the
    known-size kernel that scales the hardware byte counters."""
    import torch

    res = {}
    src = torch.ones(1 << 26, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    ms = measure(lambda: dst.copy_(src), 20)
    res["reference: device copy 256 MiB (torch copy_)"] = {"us": round(ms * 1e3, 2),
                                                          "GB/s": round(8 * (1 << 26) / ms / 1e6, 1)}
    del src, dst
    return res


def vendor_scan_reference(synth):
    """Reference only: the framework's own device scan (torch.cumsum, int32
    in and out) on the step's
    scan input, 2^26 int32 U[0,100]; 8 bytes per element."""
    import torch

    n = 1 << 26
    x = to_dev(synth.uniform_int32(synth.SEED_SCAN, n, 0, 100))
    y = torch.empty_like(x)
    ms = measure(lambda: torch.cumsum(x, 0, dtype=torch.int32, out=y), 20)
    res = {"reference: torch.cumsum int32 2^26": {"us": round(ms * 1e3, 2), "GB/s": round(8 * n / ms / 1e6, 1),
                                                  "frac_hbm": round(8 * n / ms / 1e6 / HBM_PEAK_GBS, 4)}}
    del x, y
    torch.cuda.empty_cache()
    return res


def scan_size_workloads(spmd, synth):
    """SCAN_I32 at the step's launch shape (512 x 128) on 2^28 and 2^30
    elements (U[0,100], generated on the device): 16 and 64 rounds of tiles
    per persistent block instead of 4, so the end of the launch, when
    blocks run out of tiles one after another, weighs less.  Timed with
    events bound to each launch's dispatch; every output is checked with
    the scan's defining identity y[i] - y[i-1] = x[i] (mod 2^32) on the
    device."""
    import torch

    res = {}
    for lg, reps in ((28, 10), (30, 4)):
        n = 1 << lg
        log(f"scan 2^{lg}")
        x = torch.empty(n, dtype=torch.int32, device="cuda")
        spmd.batch.synth_uniform_i32(x, synth.SEED_SCAN, 0, 100)
        y = torch.empty_like(x)
        grid = spmd.ops.scan_grid(n, SCAN_BLOCK, SCAN_ITEMS)
        ws = spmd.ops.workspace(spmd.SCAN_I32, grid, SCAN_BLOCK, n)
        for _ in range(2):
            spmd.ops.scan_i32(x, SCAN_BLOCK, SCAN_ITEMS, y=y, ws=ws)
        spans = []
        for _ in range(reps):
            ev = spmd.timing_events(2)
            spmd.ops.scan_i32(x, SCAN_BLOCK, SCAN_ITEMS, y=y, ws=ws, events=(ev[0], ev[1]))
            spans.append(ev)
        torch.cuda.synchronize()
        spmd.sync()
        ok = bool(y[0].item() == x[0].item()) and bool(torch.equal(y[1:] - y[:-1], x[1:]))
        assert ok, f"scan 2^{lg}: y[i] - y[i-1] != x[i]"
        ms = sorted(a.elapsed_time(b) for a, b in spans)[reps // 2]
        b = 8 * n
        res[f"scan_i32 2^{lg} b{SCAN_BLOCK} i{SCAN_ITEMS}"] = {
            "us": round(ms * 1e3, 2), "GB/s": round(b / ms / 1e6, 1), "frac_hbm": round(b / ms / 1e6 / HBM_PEAK_GBS, 4),
            "timing": f"median of {reps} launches, HIP events bound to each launch's dispatch", "checked": ok}
        del x, y, ws
        torch.cuda.empty_cache()
    return res


def reduce_workloads(spmd, synth):
    """REDUCE_I32: the 2^20 configuration (grid 4096, block 256, 1 KiB LDS)
    and the same class from 2^24 to 2^30 elements under a cold cache."""
    import torch

    res = {}
    log("reduce 2^20")
    n = 1 << 20
    x = to_dev(synth.uniform_int32(synth.SEED_REDUCE, n, -1000, 1000))
    p = torch.empty(4096, dtype=torch.int32, device="cuda")
    o = torch.empty(1, dtype=torch.int32, device="cuda")
    wsr = spmd.ops.workspace(spmd.REDUCE_I32, 4096, 256, n)
    ms = measure(lambda: spmd.ops.reduce_i32(x, 4096, 256, p, o, wsr), 50)
    b = 4 * n + 4 * 4096 + 4
    res["reduce_i32 2^20 g4096 b256"] = {"us": round(ms * 1e3, 2), "GB/s": round(b / ms / 1e6, 1),
                                        "frac_hbm": round(b / ms / 1e6 / HBM_PEAK_GBS, 4),
                                        "timing": "events around each host launch"}
    # the same launches replayed from a captured graph: device time without host launch cost
    expect = int(synth.uniform_int32(synth.SEED_REDUCE, n, -1000, 1000).astype(np.int64).sum())
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(3):
            spmd.ops.reduce_i32(x, 4096, 256, p, o, wsr)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    per_graph = 20
    with torch.cuda.graph(graph):
        for _ in range(per_graph):
            spmd.ops.reduce_i32(x, 4096, 256, p, o, wsr)
    for _ in range(3):  # every replay gives the eager result
        o.fill_(0)
        graph.replay()
        torch.cuda.synchronize()
        assert int(o.cpu()[0]) == expect
    ms = measure(graph.replay, 20) / per_graph
    res["reduce_i32 2^20 g4096 b256 (graph replay)"] = {
        "us": round(ms * 1e3, 2), "GB/s": round(b / ms / 1e6, 1), "frac_hbm": round(b / ms / 1e6 / HBM_PEAK_GBS, 4),
        "timing": f"one graph of {per_graph} launches, median replay / {per_graph}"}
    del graph
    del x
    # the same class where HBM, not launch latency, decides: 2^24 (64 MiB) .. 2^30 (4 GiB)
    for lg in (24, 26, 28, 30):
        n = 1 << lg
        log(f"reduce 2^{lg}")
        # cold cache: rotate over copies totalling more than 1 GiB (4x the 256 MB cache)
        copies = max(1, -(-(2 << 30) // (4 * n)))
        xs_r = [torch.ones(n, dtype=torch.int32, device="cuda") for _ in range(copies)]
        # one launch per copy in a captured graph (at least 8): device time only
        per_graph = max(8, copies)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            spmd.ops.reduce_i32(xs_r[0], 4096, 256, p, o, wsr)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            for k in range(per_graph):
                spmd.ops.reduce_i32(xs_r[k % copies], 4096, 256, p, o, wsr)
        ms = measure(graph.replay, 5, warmup=1) / per_graph
        want = n % 2**32 - (2**32 if n % 2**32 >= 2**31 else 0)
        o.fill_(0)
        graph.replay()
        torch.cuda.synchronize()
        assert int(o.cpu()[0]) == want
        b = 4 * n + 4 * 4096 + 4
        res[f"reduce_i32 2^{lg} g4096 b256"] = {"us": round(ms * 1e3, 2), "GB/s": round(b / ms / 1e6, 1),
                                              "frac_hbm": round(b / ms / 1e6 / HBM_PEAK_GBS, 4),
                                              "input_copies_rotated": copies,
                                              "timing": f"graph of {per_graph} launches, median replay / {per_graph}"}
        del graph, xs_r
        torch.cuda.empty_cache()
    return res


def jacobi_workloads(spmd, synth):
    """JACOBI5_F32: 8192^2 fp32, 100 sweeps, with the configured 16 x 16
    blocks and with 64 x 4 blocks of 4 cells."""
    import torch

    res = {}
    nn, sweeps = 8192, 100
    u = to_dev(synth.uniform_f32(synth.SEED_JACOBI, nn * nn).reshape(nn, nn))
    a, bb = u.clone(), torch.empty_like(u)
    for blk, cells in (((16, 16), 1), ((64, 4), 4)):
        log(f"jacobi {blk} x{cells}")

        def run():
            src, dst = a, bb
            for _ in range(sweeps):
                spmd.ops.jacobi5_f32(src, dst, blk, cells)
                src, dst = dst, src

        ms = measure(run, 3, warmup=1) / sweeps
        byt = 8 * nn * nn
        res[jacobi_key(blk, cells)] = {
            "us": round(ms * 1e3, 2), "GB/s": round(byt / ms / 1e6, 1),
            "frac_hbm": round(byt / ms / 1e6 / HBM_PEAK_GBS, 4)}
    # JACOBI5T_F32: the same 100 sweeps, S fused per launch (temporal
    # blocking, a roofline-raising variant reported apart from the
    # configured shape).  GB/s counts the algorithmic 8 B per cell per sweep,
    # so it can exceed what HBM moves; "hbm_bytes_per_sweep" is what a launch
    # must move (its halo-inclusive tile reads plus the interior writes),
    # divided by S.
    for per in (2, 4, 8):
        log(f"jacobi fused x{per}")

        def run_fused():
            src, dst = a, bb
            left = sweeps
            while left:
                k = min(per, left)
                spmd.ops.jacobi5t_f32(src, k, dst)
                src, dst = dst, src
                left -= k

        ms = measure(run_fused, 3, warmup=1) / sweeps
        byt = 8 * nn * nn
        halo = 4 if per <= 4 else 8
        moved = 4 * nn * nn * (256 * (64 + 2 * halo) / ((256 - 2 * halo) * 64) + 1) / per
        res[f"jacobi5t_f32 8192^2 {per} sweeps per launch (per sweep, 100 sweeps)"] = {
            "us": round(ms * 1e3, 2), "GB/s_algorithmic": round(byt / ms / 1e6, 1),
            "hbm_bytes_per_sweep": int(moved), "GB/s_hbm_moved": round(moved / ms / 1e6, 1),
            "speedup_vs_one_sweep_per_launch": None}
    base = res[jacobi_key((16, 16), 1)]["us"]
    for k, v in res.items():
        if k.startswith("jacobi5t"):
            v["speedup_vs_one_sweep_per_launch"] = round(base / v["us"], 2)
    del u, a, bb
    torch.cuda.empty_cache()
    return res


def jacobi_key(blk, cells):
    """Record name of a one-sweep Jacobi launch: the launched block shape and
    cells per thread, and the physical tile it runs as (the blocks of one
    block row are fetched 256 columns at a time as a 64 x 4 workgroup)."""
    rows = blk[1] * cells
    phys = f", runs as 256-column tiles of {rows} rows on 64x4 workgroups" if 4 <= rows <= 64 else ""
    return f"jacobi5_f32 8192^2 block{blk[0]}x{blk[1]} c{cells}{phys} (per sweep, 100 sweeps)"


def chain_workloads(spmd, synth):
    """100 dependent Jacobi sweeps (each reads the previous one's output):
    one spmd_launch per sweep from the host, the same launches captured in a
    graph, and one batch of 100 instances with dependencies
    (spmd_batch_create_dep), replayed from a graph -- once with every sweep
    as its own grid (bpf 0) and once through the persistent queue."""
    import torch

    res = {}
    sweeps = 100
    for nn in (1024, 8192):
        u_h = synth.uniform_f32(synth.SEED_JACOBI, nn * nn).reshape(nn, nn)
        u0 = to_dev(u_h)
        bufs = [u0.clone(), torch.empty_like(u0)]

        def launches():
            for t in range(sweeps):
                spmd.ops.jacobi5_f32(bufs[t % 2], bufs[(t + 1) % 2], (16, 16), 1)

        log(f"jacobi chain {nn}^2 x {sweeps}")
        ms_host = measure(launches, 3, warmup=1)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            launches()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            launches()
        ms_graph = measure(g.replay, 3, warmup=1)
        bufs[0].copy_(u0)
        g.replay()
        torch.cuda.synchronize()
        ref = bufs[sweeps % 2].clone()
        del g
        items = [(spmd.JACOBI5_F32, nn, nn, 256, bufs[t % 2], bufs[(t + 1) % 2]) for t in range(sweeps)]
        deps = [None] + list(range(sweeps - 1))
        rec = {"ms_one_launch_per_sweep": round(ms_host, 3), "ms_launches_captured_graph": round(ms_graph, 3)}
        same = True
        for name, sched in (("own_grids", (256, 4, 0)), ("queue", (512, 4, 8))):
            b = spmd.batch.Batch(items, [sched] * sweeps, deps=deps)
            bufs[0].copy_(u0)
            b.graph_launch()
            spmd.sync()
            same = same and bool(torch.equal(ref, bufs[sweeps % 2]))
            ms = measure(b.graph_launch, 3, warmup=1)
            spmd.sync()
            b.close()
            rec[f"ms_dependent_batch_{name}"] = round(ms, 3)
            rec[f"schedule_{name}"] = list(sched)
        rec["GB/s_dependent_batch_own_grids"] = round(8 * nn * nn * sweeps / rec["ms_dependent_batch_own_grids"] / 1e6, 1)
        rec["outputs_identical"] = same
        res[f"jacobi chain {nn}^2 x {sweeps} sweeps"] = rec
        del bufs, u0
        torch.cuda.empty_cache()
    return res


def hist_contention_workloads(spmd, synth):
    """The histogram at the step's shape (2^27 keys, grid 256, block 1024)
    under LDS-atomic contention: bounded Zipf exponents 0 (uniform) to 3,
    hot bins in place or sent through the seeded bin permutation, and every
    key in one bin."""
    import torch

    from paper_2206_07896_amd import batch as B

    n = HIST_N
    keys = torch.empty(n, dtype=torch.int32, device="cuda")
    hist = torch.empty(256, dtype=torch.int32, device="cuda")
    perm = torch.from_numpy(synth.bin_permutation().astype(np.int32)).cuda()
    res = {}
    keys.zero_()
    measure(lambda: spmd.ops.hist256_u32(keys, HIST_GRID, HIST_BLOCK, hist=hist), 10, warmup=5)  # settle clocks
    for alpha in (0.0, 1.1, 2.0, 3.0, "one"):
        for permuted in ((False, True) if alpha != "one" else (False,)):
            if alpha == "one":
                keys.fill_(7)
            else:
                cdf = torch.from_numpy(synth.zipf_cdf(alpha, 256)).cuda()
                B.synth_zipf_u32(keys, synth.SEED_HIST, cdf)
                if permuted:
                    keys.copy_(perm[keys.long()])
            torch.cuda.synchronize()
            ms = measure(lambda: spmd.ops.hist256_u32(keys, HIST_GRID, HIST_BLOCK, hist=hist), 10, warmup=3)
            assert int(hist.cpu().numpy().view(np.uint32).astype(np.int64).sum()) == n
            name = "one bin" if alpha == "one" else f"zipf{alpha}" + (" permuted" if permuted else "")
            gbs = 4 * n / ms / 1e6
            res[f"hist contention: hist256_u32 2^27 {name} g{HIST_GRID} b{HIST_BLOCK}"] = {
                "us": round(ms * 1e3, 2), "GB/s": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)}
    del keys
    torch.cuda.empty_cache()
    return res


def compact_workloads(spmd, synth):
    """COMPACT_I32: 2^26 int32 U[-1000,1000] (seed of the scan input), t = 0
    (about half kept), blockDim 256 with 16 items, inputs rotated over two
    copies; bytes = 4 per element read + 4 per element kept + the count."""
    import torch

    res = {}
    n = 1 << 26
    x_h = synth.uniform_int32(synth.SEED_SCAN, n, -1000, 1000)
    xs = [to_dev(x_h), to_dev(x_h)]
    y = torch.empty_like(xs[0])
    count = torch.zeros(1, dtype=torch.int32, device="cuda")
    for block, items in ((1024, 32), (512, 32)):
        grid = spmd.ops.compact_grid(n, block, items)
        ws = spmd.ops.workspace(spmd.COMPACT_I32, grid, block, n)
        log(f"compact 2^26 b{block} i{items}")
        turn = [0]

        def run():
            spmd.ops.compact_i32(xs[turn[0] & 1], 0, block, items, y=y, count=count, ws=ws)
            turn[0] += 1

        ms = measure(run, 20)
        m = int(count.cpu()[0])
        assert m == int(np.count_nonzero(x_h > 0))
        byts = 4 * n + 4 * m + 4
        res[f"compact_i32 2^26 t=0 b{block} i{items}"] = {"us": round(ms * 1e3, 2), "kept": m,
                                                          "GB/s": round(byts / ms / 1e6, 1),
                                                          "frac_hbm": round(byts / ms / 1e6 / HBM_PEAK_GBS, 4)}
    # reference only: the framework's selection (torch.masked_select) on the same input, same bytes
    ms = measure(lambda: torch.masked_select(xs[0], xs[0] > 0), 20)
    res["reference: torch.masked_select 2^26 t=0"] = {"us": round(ms * 1e3, 2), "GB/s": round(byts / ms / 1e6, 1)}
    del xs, y
    torch.cuda.empty_cache()
    return res


def gemm_workloads(spmd, synth, reps=10, n=4096):
    """C = A B, n^3 fp32 N(0,1) (4096 by default), at the configured 64 x 64
    tiles and at 128 x 128 and 256 x 256 (the larger tiles reported apart
    from the configured shape)."""
    import torch

    res = {}
    A = to_dev(synth.normal_f32(synth.SEED_GEMM, n * n).reshape(n, n))
    B = to_dev(synth.normal_f32(synth.SEED_GEMM + 1, n * n).reshape(n, n))
    C = torch.empty_like(A)
    # The chip's clock ramps over the first few hundred ms of MFMA load; the
    # first configuration measured cold reads 10-15% low.  Settle it first.
    for _ in range(max(4, int(2e13 // (2 * n**3)))):
        spmd.ops.gemm_f32(A, B, C, 128)
    spmd.sync()
    for tile in (64, 128, 256):
        log(f"gemm tile {tile}")
        ms = measure(lambda: spmd.ops.gemm_f32(A, B, C, tile), reps)
        tf = 2 * n**3 / (ms * 1e-3) / 1e12
        res[f"gemm_f32 {n}^3 tile{tile}"] = {"us": round(ms * 1e3, 2), "TFLOP/s": round(tf, 2),
                                              "frac_mfma_fp32": round(tf / FP32_MFMA_PEAK_TFS, 4)}
    spmd.sync()
    # reference only: the vendor library GEMM (torch.matmul, fp32 without TF32) on the same operands
    torch.backends.cuda.matmul.allow_tf32 = False
    ms = measure(lambda: torch.matmul(A, B, out=C), reps)
    tf = 2 * n**3 / (ms * 1e-3) / 1e12
    res[f"reference: torch.matmul fp32 {n}^3"] = {"us": round(ms * 1e3, 2), "TFLOP/s": round(tf, 2),
                                                  "frac_mfma_fp32": round(tf / FP32_MFMA_PEAK_TFS, 4)}
    return res


def mixed_queue(spmd, count, reps=10):
    """Mixed launches: `count` instances (class uniform over reduce, scan,
    hist, jacobi; n = round(2^U), U ~ U[10, 22]; blockDim uniform over
    64..512), each written as a CUDA launch with its blockDim and 4 items
    per thread.  Compared on the same inputs:
      * one launch per instance from a host loop (hardware block dispatch),
        the baseline;
      * the persistent queue replayed from a hipGraph with the same
        schedule and the paper's average coarse-grained fetching;
      * the persistent queue replayed from a hipGraph with the schedule the
        shipped cost model picks (when the package holds one).
    Outputs must agree bit for bit."""
    import torch

    from paper_2206_07896_amd import learned as L
    from paper_2206_07896_amd import workload as W

    log(f"mixed queue: {count} instances")
    specs = W.mixed_specs(count)
    data = W.MixedData(specs)
    heur = W.as_launched_schedules(specs)
    b = spmd.batch.Batch(data.items(), heur)
    st = b.stats()
    data.outputs.fill_(-1)  # same padding bytes between instances in every run
    b.graph_launch()
    spmd.sync()
    ref = data.outputs.clone()
    data.outputs.fill_(-1)
    b.launch_each()
    spmd.sync()
    same = bool(torch.equal(ref, data.outputs))
    t_graph = measure(b.graph_launch, reps, warmup=2)
    t_each = measure(b.launch_each, max(3, reps // 2), warmup=1)
    spmd.sync()
    # the same one-launch-per-instance sequence captured once into a graph:
    # the dispatch cost of separate grids without the host's launch cost
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        b.launch_each()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    each_graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(each_graph):
        b.launch_each()
    for _ in range(2):  # every replay gives the eager result
        data.outputs.fill_(-1)
        each_graph.replay()
        torch.cuda.synchronize()
        same = same and bool(torch.equal(ref, data.outputs))
    t_each_graph = measure(each_graph.replay, 5, warmup=1)
    del each_graph
    spmd.sync()
    b.close()
    gbytes = data.total_bytes / 1e9
    res = {
        "instances": count,
        "logical_blocks": st["blocks"],
        "kernel_launches_one_by_one": st["each_launches"],
        "ms_one_by_one": round(t_each, 3),
        "launches_per_s_one_by_one": round(count / (t_each * 1e-3), 1),
        "ms_one_by_one_captured_graph": round(t_each_graph, 3),
        "heuristic": {"schedule": "blockDim as launched, 4 items/thread, average coarse-grained fetching "
                                  "ceil(blocks/pool)",
                      "chunks": st["chunks"], "kernel_launches": st["persistent_launches"],
                      "ms_graph": round(t_graph, 3),
                      "launches_per_s": round(count / (t_graph * 1e-3), 1),
                      "speedup_vs_one_by_one": round(t_each / t_graph, 3),
                      "GB/s": round(gbytes / (t_graph * 1e-3), 1)},
    }
    log(f"mixed: one-by-one {t_each:.2f} ms (captured {t_each_graph:.2f} ms), heuristic graph {t_graph:.2f} ms")
    model = L.load_default()
    if model is not None:
        # per launch: the least predicted time of each launch alone; batch-
        # aware: the fewest chunks within SPMD_BATCH_SLACK of it (the choice
        # spmd_launch_batch makes in SPMD_SCHED_LEARNED mode)
        for key, slack, what in (("learned", None, "cost model, least predicted time per launch, no fallback"),
                                 ("learned_batch", model.slack,
                                  f"cost model, batch-aware: fewest chunks within {model.slack:.0%} of the least "
                                  "predicted time (the model's slack, chosen on held-out launches), no fallback")):
            choice, _, sd = model.choose(specs, slack=slack)
            sched = [L.CANDIDATES[j] for j in choice]
            bl = spmd.batch.Batch(data.items(), sched)
            stl = bl.stats()
            data.outputs.fill_(-1)
            bl.graph_launch()
            spmd.sync()
            same = same and bool(torch.equal(ref, data.outputs))
            t_l = measure(bl.graph_launch, reps, warmup=2)
            spmd.sync()
            bl.close()
            res[key] = {"schedule": what,
                        "chunks": stl["chunks"], "kernel_launches": stl["persistent_launches"],
                        "ms_graph": round(t_l, 3),
                        "launches_per_s": round(count / (t_l * 1e-3), 1),
                        "speedup_vs_one_by_one": round(t_each / t_l, 3),
                        "speedup_vs_one_by_one_captured_graph": round(t_each_graph / t_l, 3),
                        "speedup_vs_heuristic": round(t_graph / t_l, 3),
                        "GB/s": round(gbytes / (t_l * 1e-3), 1),
                        "frac_hbm": round(gbytes / (t_l * 1e-3) / HBM_PEAK_GBS, 4),
                        "low_confidence_launches": int((sd > model.tau).sum())}
            log(f"mixed: {key} graph {t_l:.2f} ms")
    res["outputs_identical"] = same
    del ref, data
    torch.cuda.empty_cache()
    return res


def source_hash(paths):
    import hashlib

    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


TRAFFIC_SOURCES = {
    "scan": ["paper_2206_07896_amd/csrc/k_scan.hip", "paper_2206_07896_amd/csrc/cls_scan.hpp",
             "paper_2206_07896_amd/csrc/warp32.hpp"],
    "hist": ["paper_2206_07896_amd/csrc/k_hist.hip", "paper_2206_07896_amd/csrc/cls_hist.hpp",
             "paper_2206_07896_amd/csrc/warp32.hpp"],
}


def measured_traffic(kernel_name):
    """HBM bytes per launch from the committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by the same counters' reading for a
    copy of known size), or None when there is none or the kernel's sources
    changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    data = json.load(open(path))
    rec = data.get(kernel_name)
    if not rec:
        return None
    cls = "scan" if kernel_name.startswith("scan") else "hist"
    if rec.get("source_hash") != source_hash(TRAFFIC_SOURCES[cls]):
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(xs_h, ks_h, step_bytes):
    """The oracle executor (thread-pool runtime of the paper, average
    coarse-grained fetching) on the same step: scan then histogram."""
    import oracle

    pool = min(16, os.cpu_count() or 1)
    log(f"cpu oracle, pool {pool}")
    # the oracle's executor holds at most 64 items per thread; the scan it
    # computes does not depend on the launch shape
    items = min(SCAN_ITEMS, 64)
    oracle.scan_i32(xs_h[:4096], SCAN_BLOCK, items, pool=pool)  # start the pool
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        oracle.scan_i32(xs_h, SCAN_BLOCK, items, pool=pool)
        oracle.hist256_u32(ks_h, HIST_GRID, HIST_BLOCK, pool=pool)
        times.append(time.perf_counter() - t0)
    t = sorted(times)[1]
    return {"value": round(step_bytes / t / 1e9, 3), "unit": "GB/s", "cores": pool, "kind": "oracle",
            "sample": f"the full step (scan 2^26 at {SCAN_BLOCK} x {items} + hist 2^27) on the oracle's thread-pool "
                      f"executor, median of 3 runs, {t:.2f} s each"}


def _median_seconds(fn, runs=3):
    ts = []
    for _ in range(runs):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    return sorted(ts)[len(ts) // 2]


def cpu_executor_baselines(mixed_count):
    """The oracle's thread-pool executor (the paper's runtime: a pool of
    workers fetching ceil(grid / pool) blocks at a time) on the other
    workloads, with the GPU figures' algorithmic denominators:
      * reduce 2^20 int32, grid 4096, block 256 (median of 5 runs);
      * one Jacobi sweep of the 8192^2 grid in 16 x 16 blocks (median of 3);
      * GEMM at 2048^3 instead of 4096^3 (one run; the executor needs
        about a minute at the full size);
      * a seeded sample of 1000 instances of the mixed workload, each as
        launched (its blockDim, 4 items per thread; stencils in 16 x 16
        blocks), one after the other.
    Each row is a baseline, not the target."""
    import oracle
    import synth

    from paper_2206_07896_amd import workload as W

    pool = min(16, os.cpu_count() or 1)
    res = {}
    x = synth.uniform_int32(synth.SEED_REDUCE, 1 << 20, -1000, 1000)
    oracle.reduce_i32(x[:4096], 16, 256, pool=pool)  # start the pool
    t = _median_seconds(lambda: oracle.reduce_i32(x, 4096, 256, pool=pool), runs=5)
    nbytes = 4 * (1 << 20) + 4 * 4096 * 2 + 4
    res["reduce_i32 2^20 g4096 b256"] = {"us": round(t * 1e6, 1), "GB/s": round(nbytes / t / 1e9, 3),
                                         "cores": pool, "runs": 5}
    u = synth.uniform_f32(synth.SEED_JACOBI, 8192 * 8192).reshape(8192, 8192)
    t = _median_seconds(lambda: oracle.jacobi5_f32(u, 16, 16, pool=pool), runs=3)
    res[jacobi_key((16, 16), 1)] = {
        "us": round(t * 1e6, 1), "GB/s": round(8 * 8192 * 8192 / t / 1e9, 3), "cores": pool,
        "sample": "one sweep, median of 3"}
    del u
    m = 2048
    A = synth.normal_f32(synth.SEED_GEMM, m * m).reshape(m, m)
    B = synth.normal_f32(synth.SEED_GEMM + 1, m * m).reshape(m, m)
    t = _median_seconds(lambda: oracle.gemm_f32(A, B, pool=pool), runs=1)
    res["gemm_f32 4096^3 tile64"] = {"us": round(t * 1e6, 1), "TFLOP/s": round(2 * m ** 3 / t / 1e12, 6),
                                     "cores": pool, "sample": "2048^3 instead of 4096^3"}
    specs = W.mixed_specs(mixed_count)
    rng = np.random.default_rng(0xC4)
    sample = [specs[i] for i in sorted(rng.choice(len(specs), min(1000, len(specs)), replace=False).tolist())]
    inputs = [W.host_input(s) for s in sample]

    def run_sample():
        for s, xi in zip(sample, inputs):
            k, bd, n = s["kid"], s["block_dim"], s["n"]
            grid = max(1, -(-n // (bd * 4)))
            if k == W.REDUCE_I32:
                oracle.reduce_i32(xi, grid, bd, pool=pool)
            elif k == W.SCAN_I32:
                oracle.scan_i32(xi, bd, 4, pool=pool)
            elif k == W.HIST256_U32:
                oracle.hist256_u32(xi, grid, bd, pool=pool)
            else:
                oracle.jacobi5_f32(xi, 16, 16, pool=pool)

    t = _median_seconds(run_sample, runs=1)
    nbytes = sum(W.algorithmic_bytes(s) for s in sample)
    res["mixed_queue"] = {"instances": len(sample), "seconds": round(t, 3),
                          "launches_per_s": round(len(sample) / t, 1), "GB/s": round(nbytes / t / 1e9, 3),
                          "cores": pool,
                          "sample": f"{len(sample)} instances drawn (seed 0xC4) from the {mixed_count}-instance workload"}
    log(f"cpu oracle executor: {json.dumps(res)}")
    return res


if __name__ == "__main__":
    main()
