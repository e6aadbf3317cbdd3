"""Synthetic mixed-launch workloads for the batched queue.

An instance is one launch of a kernel class: class uniform over REDUCE,
SCAN, HIST and JACOBI; size n = round(2^U) with U uniform on
[log2_lo, log2_hi] (JACOBI: one sweep of a round(sqrt(n)) square grid);
blockDim uniform over {64, 128, 256, 512}.  Instance i draws its input from
the seed (seed ^ i): REDUCE uniform int32 [-1000, 1000], SCAN uniform
int32 [0, 100], HIST Zipf(1.1) keys over 256 bins, JACOBI uniform fp32
[0, 1).  Inputs are generated on the device by the library's counter-based
generator, which yields the same values as the host generator ``synth``.
"""

from __future__ import annotations

import numpy as np
import torch

import synth

from . import HIST256_U32, JACOBI5_F32, REDUCE_I32, SCAN_I32
from . import batch as B

KIND_IDS = (REDUCE_I32, SCAN_I32, HIST256_U32, JACOBI5_F32)
KIND_NAMES = {REDUCE_I32: "reduce", SCAN_I32: "scan", HIST256_U32: "hist", JACOBI5_F32: "jacobi"}
BLOCK_DIMS = (64, 128, 256, 512)
ALIGN = 64  # elements (256 bytes) between instance buffers


def mixed_specs(count: int, seed: int = synth.SEED_BATCH, log2_lo: float = 10.0, log2_hi: float = 22.0):
    u = synth.uniform_unit_f64(seed, 3 * count).reshape(count, 3)
    specs = []
    for i in range(count):
        kid = KIND_IDS[min(3, int(u[i, 0] * 4))]
        n = int(round(2.0 ** (log2_lo + (log2_hi - log2_lo) * u[i, 1])))
        bd = BLOCK_DIMS[min(3, int(u[i, 2] * 4))]
        if kid == JACOBI5_F32:
            side = max(1, int(round(np.sqrt(n))))
            nx, ny = side, side
            n = side * side
        else:
            nx, ny = n, 1
        specs.append({"kid": kid, "n": n, "nx": nx, "ny": ny, "block_dim": bd, "seed": seed ^ i})
    return specs


def algorithmic_bytes(spec) -> int:
    k, n = spec["kid"], spec["n"]
    if k == REDUCE_I32:
        return 4 * n + 4
    if k == SCAN_I32:
        return 8 * n
    if k == HIST256_U32:
        return 4 * n + 1024
    return 8 * n


def _pad(n: int) -> int:
    return max(ALIGN, -(-n // ALIGN) * ALIGN)


class MixedData:
    """Device buffers of a list of specs: one input and one output arena,
    each instance at a 256-byte aligned offset, inputs filled on the
    device."""

    def __init__(self, specs, device="cuda"):
        self.specs = specs
        in_off, out_off = [], []
        ti = to = 0
        for s in specs:
            in_off.append(ti)
            ti += _pad(s["n"])
            out_elems = {REDUCE_I32: 1, SCAN_I32: s["n"], HIST256_U32: 256, JACOBI5_F32: s["n"]}[s["kid"]]
            out_off.append(to)
            to += _pad(out_elems)
        self.inputs = torch.empty(ti, dtype=torch.int32, device=device)
        self.outputs = torch.zeros(to, dtype=torch.int32, device=device)
        self.in_off, self.out_off = in_off, out_off
        cdf = torch.from_numpy(synth.zipf_cdf(1.1, 256)).to(device)
        for s, o in zip(specs, in_off):
            t = self.inputs[o:o + s["n"]]
            k = s["kid"]
            if k == REDUCE_I32:
                B.synth_uniform_i32(t, s["seed"], -1000, 1000)
            elif k == SCAN_I32:
                B.synth_uniform_i32(t, s["seed"], 0, 100)
            elif k == HIST256_U32:
                B.synth_zipf_u32(t, s["seed"], cdf)
            else:
                B.synth_uniform_f32(t.view(torch.float32), s["seed"])
        self.total_bytes = sum(algorithmic_bytes(s) for s in specs)

    def input_of(self, i):
        s = self.specs[i]
        t = self.inputs[self.in_off[i]:self.in_off[i] + s["n"]]
        return t.view(torch.float32).view(s["ny"], s["nx"]) if s["kid"] == JACOBI5_F32 else t

    def output_of(self, i):
        s = self.specs[i]
        k = s["kid"]
        n = {REDUCE_I32: 1, SCAN_I32: s["n"], HIST256_U32: 256, JACOBI5_F32: s["n"]}[k]
        t = self.outputs[self.out_off[i]:self.out_off[i] + n]
        return t.view(torch.float32).view(s["ny"], s["nx"]) if k == JACOBI5_F32 else t

    def items(self):
        out = []
        for i, s in enumerate(self.specs):
            out.append((s["kid"], s["nx"], s["ny"], s["block_dim"], self.input_of(i), self.output_of(i)))
        return out

    def host_input(self, i):
        """The same input regenerated on the host (for checks)."""
        return host_input(self.specs[i])


def host_input(s):
    """Input of spec `s` generated on the host (the values MixedData fills on
    the device)."""
    k = s["kid"]
    if k == REDUCE_I32:
        return synth.uniform_int32(s["seed"], s["n"], -1000, 1000)
    if k == SCAN_I32:
        return synth.uniform_int32(s["seed"], s["n"], 0, 100)
    if k == HIST256_U32:
        return synth.zipf_u32(s["seed"], s["n"])
    return synth.uniform_f32(s["seed"], s["n"]).reshape(s["ny"], s["nx"])


def as_launched_schedules(specs, items: int = 4, workers_per_cu: int = 0):
    """Each instance with its own blockDim, `items` per thread, and the
    paper's average coarse-grained fetching: ceil(blocks / pool) blocks per
    fetch, pool = the persistent workers of its (class, block size) queue."""
    pools = {(k, b): B.pool_size(k, b, workers_per_cu) for k in KIND_IDS for b in BLOCK_DIMS}
    out = []
    for s in specs:
        it = min(items, 8) if s["kid"] == JACOBI5_F32 else items
        nb = B.item_blocks(s["kid"], s["nx"], s["ny"], s["block_dim"], it)
        out.append((s["block_dim"], it, B.average_bpf(nb, pools[(s["kid"], s["block_dim"])])))
    return out
