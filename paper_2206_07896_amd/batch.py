"""Binding of spmd_batch.h (persistent block queue) and spmd_synth.h
(device-side seeded inputs).  Argument marshalling only."""

from __future__ import annotations

import ctypes

import torch

from . import SpmdError, _check, _lib, _stream_handle

_P = ctypes.c_void_p
_U32 = ctypes.c_uint32
_U64 = ctypes.c_uint64


class Schedule(ctypes.Structure):
    _fields_ = [("block", _U32), ("items", _U32), ("bpf", _U32)]


class BatchItem(ctypes.Structure):
    _fields_ = [("kernel_id", ctypes.c_int32), ("n", _U32), ("ny", _U32), ("block_dim", _U32), ("in_", _P),
                ("out", _P)]


_lib.spmd_batch_item_blocks.argtypes = [ctypes.POINTER(BatchItem), ctypes.POINTER(Schedule)]
_lib.spmd_batch_item_blocks.restype = _U64
_lib.spmd_batch_workspace_size.argtypes = [ctypes.POINTER(BatchItem), ctypes.POINTER(Schedule), ctypes.c_int]
_lib.spmd_batch_workspace_size.restype = ctypes.c_size_t
_lib.spmd_batch_create.argtypes = [ctypes.POINTER(BatchItem), ctypes.POINTER(Schedule), ctypes.c_int, _P,
                                   ctypes.c_size_t, _U32, ctypes.POINTER(_P)]
_lib.spmd_batch_create.restype = ctypes.c_int
_lib.spmd_batch_workspace_size_dep.argtypes = [ctypes.POINTER(BatchItem), ctypes.POINTER(Schedule), _P, ctypes.c_int]
_lib.spmd_batch_workspace_size_dep.restype = ctypes.c_size_t
_lib.spmd_batch_create_dep.argtypes = [ctypes.POINTER(BatchItem), ctypes.POINTER(Schedule), _P, ctypes.c_int, _P,
                                       ctypes.c_size_t, _U32, ctypes.POINTER(_P)]
_lib.spmd_batch_create_dep.restype = ctypes.c_int
NO_DEP = 0xFFFFFFFF
for _f in ("spmd_batch_launch", "spmd_batch_graph_launch", "spmd_batch_launch_each"):
    getattr(_lib, _f).argtypes = [_P, _P]
    getattr(_lib, _f).restype = ctypes.c_int
_lib.spmd_batch_stats.argtypes = [_P, ctypes.POINTER(_U64), ctypes.POINTER(_U64), ctypes.POINTER(_U32),
                                  ctypes.POINTER(_U32)]
_lib.spmd_batch_stats.restype = ctypes.c_int
_lib.spmd_batch_pool_size.argtypes = [ctypes.c_int, _U32, _U32, ctypes.POINTER(_U32)]
_lib.spmd_batch_pool_size.restype = ctypes.c_int
_lib.spmd_batch_destroy.argtypes = [_P]
_lib.spmd_batch_destroy.restype = ctypes.c_int

_lib.spmd_synth_key.argtypes = [_U64]
_lib.spmd_synth_key.restype = _U64
_lib.spmd_synth_uniform_i32.argtypes = [_P, _U64, _U64, _U64, ctypes.c_int32, ctypes.c_int32, _P]
_lib.spmd_synth_uniform_f32.argtypes = [_P, _U64, _U64, _U64, _P]
_lib.spmd_synth_raw_u32.argtypes = [_P, _U64, _U64, _U64, _P]
_lib.spmd_synth_zipf_u32.argtypes = [_P, _U64, _U64, _U64, _P, _U32, _P]
for _f in ("spmd_synth_uniform_i32", "spmd_synth_uniform_f32", "spmd_synth_raw_u32", "spmd_synth_zipf_u32"):
    getattr(_lib, _f).restype = ctypes.c_int


def _ptr(t):
    return 0 if t is None else (t if isinstance(t, int) else t.data_ptr())


def item_blocks(kernel_id: int, n: int, ny: int, block: int, items: int, bpf: int = 1) -> int:
    it = BatchItem(kernel_id, n, ny, block, None, None)
    s = Schedule(block, items, bpf)
    return int(_lib.spmd_batch_item_blocks(ctypes.byref(it), ctypes.byref(s)))


def pool_size(kernel_id: int, block: int, workers_per_cu: int = 0) -> int:
    """Persistent workgroups of `block` threads a batch runs for a class."""
    v = _U32()
    _check(_lib.spmd_batch_pool_size(kernel_id, block, workers_per_cu, ctypes.byref(v)), "spmd_batch_pool_size")
    return v.value


def average_bpf(blocks: int, pool: int) -> int:
    """The paper's average coarse-grained fetching: ceil(grid / pool)."""
    return max(1, -(-blocks // max(1, pool)))


class Batch:
    """A prepared batch: items (kernel_id, n, ny, block_dim, in, out) with
    one schedule (block, items, bpf) each.  Tensors must stay alive while
    the batch is used; the batch keeps references to them."""

    def __init__(self, items, schedules, workers_per_cu: int = 0, device=None, deps=None):
        """deps: optional list, deps[i] = index of an earlier instance whose
        output instance i reads, or None (spmd_batch_create_dep)."""
        n = len(items)
        if n == 0 or len(schedules) != n:
            raise SpmdError(-4, "Batch: need one schedule per item")
        dep_arr = None
        if deps is not None:
            if len(deps) != n:
                raise SpmdError(-4, "Batch: need one dependency entry per item")
            dep_arr = (_U32 * n)(*[NO_DEP if d is None else int(d) for d in deps])
        self._keep = []
        arr = (BatchItem * n)()
        sch = (Schedule * n)()
        for i, (kid, nn, ny, bd, tin, tout) in enumerate(items):
            arr[i] = BatchItem(int(kid), int(nn), int(ny), int(bd), _ptr(tin), _ptr(tout))
            self._keep += [tin, tout]
        for i, (b, it, bpf) in enumerate(schedules):
            sch[i] = Schedule(int(b), int(it), int(bpf))
        size = int(_lib.spmd_batch_workspace_size_dep(arr, sch, dep_arr, n))
        if size == 0:  # the plan is invalid: create reports why before it looks at the workspace
            rc = _lib.spmd_batch_create_dep(arr, sch, dep_arr, n, None, 0, workers_per_cu, ctypes.byref(_P()))
            raise SpmdError(rc if rc else -2, "spmd_batch_create (invalid items, schedules or dependencies)")
        raw = torch.empty(size + 256, dtype=torch.uint8, device=device or "cuda")
        off = (-raw.data_ptr()) % 256
        self.workspace = raw[off:off + size]
        self._raw = raw
        h = _P()
        _check(_lib.spmd_batch_create_dep(arr, sch, dep_arr, n, self.workspace.data_ptr(), size, workers_per_cu,
                                          ctypes.byref(h)), "spmd_batch_create")
        self._deps = dep_arr
        self._h = h
        self.n = n
        self._items = arr
        self._sched = sch

    def launch(self, stream=None):
        _check(_lib.spmd_batch_launch(self._h, _stream_handle(stream)), "spmd_batch_launch")

    def graph_launch(self, stream=None):
        _check(_lib.spmd_batch_graph_launch(self._h, _stream_handle(stream)), "spmd_batch_graph_launch")

    def launch_each(self, stream=None):
        _check(_lib.spmd_batch_launch_each(self._h, _stream_handle(stream)), "spmd_batch_launch_each")

    def stats(self):
        b, c = _U64(), _U64()
        p, e = _U32(), _U32()
        _check(_lib.spmd_batch_stats(self._h, ctypes.byref(b), ctypes.byref(c), ctypes.byref(p), ctypes.byref(e)),
               "spmd_batch_stats")
        return {"blocks": b.value, "chunks": c.value, "persistent_launches": p.value, "each_launches": e.value}

    def close(self):
        if getattr(self, "_h", None):
            _lib.spmd_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# device-side seeded inputs (same streams as the host generator)
# ---------------------------------------------------------------------------

def synth_key(seed: int) -> int:
    return int(_lib.spmd_synth_key(seed & 0xFFFFFFFFFFFFFFFF))


def synth_uniform_i32(out: torch.Tensor, seed: int, lo: int, hi: int, start: int = 0, stream=None):
    _check(_lib.spmd_synth_uniform_i32(out.data_ptr(), out.numel(), seed, start, lo, hi, _stream_handle(stream)),
           "spmd_synth_uniform_i32")
    return out


def synth_uniform_f32(out: torch.Tensor, seed: int, start: int = 0, stream=None):
    _check(_lib.spmd_synth_uniform_f32(out.data_ptr(), out.numel(), seed, start, _stream_handle(stream)),
           "spmd_synth_uniform_f32")
    return out


def synth_raw_u32(out: torch.Tensor, seed: int, start: int = 0, stream=None):
    _check(_lib.spmd_synth_raw_u32(out.data_ptr(), out.numel(), seed, start, _stream_handle(stream)),
           "spmd_synth_raw_u32")
    return out


def synth_zipf_u32(out: torch.Tensor, seed: int, cdf: torch.Tensor, start: int = 0, stream=None):
    assert cdf.dtype == torch.float64 and cdf.is_cuda
    _check(_lib.spmd_synth_zipf_u32(out.data_ptr(), out.numel(), seed, start, cdf.data_ptr(), cdf.numel(),
                                    _stream_handle(stream)), "spmd_synth_zipf_u32")
    return out


# ---- CUDA-style launch descriptors run as one batch (spmd_launch_batch) ----

SCHED_AS_LAUNCHED = 0
SCHED_LEARNED = 1


class LaunchDesc(ctypes.Structure):
    _fields_ = [("kernel_id", ctypes.c_int32), ("grid", _U32 * 3), ("block", _U32 * 3), ("dyn_shmem", _U32),
                ("args", ctypes.POINTER(_P))]


class BatchReport(ctypes.Structure):
    _fields_ = [("launches", _U32), ("by_model", _U32), ("tuned", _U32), ("cached", _U32)]


_lib.spmd_launch_batch_workspace_size.argtypes = [ctypes.POINTER(LaunchDesc), ctypes.c_int]
_lib.spmd_launch_batch_workspace_size.restype = ctypes.c_size_t
_lib.spmd_launch_batch.argtypes = [ctypes.POINTER(LaunchDesc), ctypes.c_int, ctypes.c_int, _P, ctypes.c_size_t, _P]
_lib.spmd_launch_batch.restype = ctypes.c_int
_lib.spmd_launch_batch_report.argtypes = [ctypes.POINTER(BatchReport)]
_lib.spmd_launch_batch_report.restype = ctypes.c_int
_lib.spmd_model_load.argtypes = [_P, _U32, _P, ctypes.c_float]
_lib.spmd_model_load.restype = ctypes.c_int
_lib.spmd_model_batch_slack.argtypes = [ctypes.c_float]
_lib.spmd_model_batch_slack.restype = ctypes.c_int
_lib.spmd_sched_candidates.argtypes = [ctypes.POINTER(Schedule), _U32]
_lib.spmd_sched_candidates.restype = _U32
_lib.spmd_sched_features.argtypes = [ctypes.POINTER(BatchItem), ctypes.POINTER(ctypes.c_float)]
_lib.spmd_sched_features.restype = ctypes.c_int


def _dims(d):
    d = tuple(d) if isinstance(d, (tuple, list)) else (d,)
    d = d + (1,) * (3 - len(d))
    return (_U32 * 3)(*map(int, d))


class _Descs:
    """Marshalled launch descriptors (kernel_id, grid, block, dyn_shmem,
    args); keeps the packed argument objects alive."""

    def __init__(self, launches):
        from . import pack_args

        self.n = len(launches)
        self.arr = (LaunchDesc * self.n)()
        self._keep = []
        for i, (kid, grid, block, shmem, args) in enumerate(launches):
            packed, keep = pack_args(kid, args)
            self._keep.append((packed, keep))
            self.arr[i] = LaunchDesc(int(kid), _dims(grid), _dims(block), int(shmem),
                                     ctypes.cast(packed, ctypes.POINTER(_P)))


def launch_batch_workspace_size(launches) -> int:
    d = _Descs(launches)
    return int(_lib.spmd_launch_batch_workspace_size(d.arr, d.n))


def launch_batch(launches, mode: int = SCHED_AS_LAUNCHED, workspace=None, stream=None):
    """Run launches [(kernel_id, grid, block, dyn_shmem, args), ...] as one
    batch; returns the workspace tensor (keep it alive until the batch is
    synchronised)."""
    d = _Descs(launches)
    size = int(_lib.spmd_launch_batch_workspace_size(d.arr, d.n))
    if size == 0:  # a launch cannot be batched: the call reports why before it looks at the workspace
        rc = _lib.spmd_launch_batch(d.arr, d.n, int(mode), None, 0, _stream_handle(stream))
        raise SpmdError(rc if rc else -2, "spmd_launch_batch (a launch cannot be batched)")
    if workspace is None or workspace.numel() < size + 256:
        workspace = torch.empty(size + 256, dtype=torch.uint8, device="cuda")
    off = (-workspace.data_ptr()) % 256
    _check(_lib.spmd_launch_batch(d.arr, d.n, int(mode), workspace.data_ptr() + off, workspace.numel() - off,
                                  _stream_handle(stream)), "spmd_launch_batch")
    return workspace


def launch_batch_report() -> dict:
    r = BatchReport()
    _check(_lib.spmd_launch_batch_report(ctypes.byref(r)), "spmd_launch_batch_report")
    return {"launches": r.launches, "by_model": r.by_model, "tuned": r.tuned, "cached": r.cached}


def model_load(params, norm, sd_threshold: float = float("inf"), slack: float | None = None) -> None:
    """Load a cost model (host arrays: [k, NPARAM] parameters, 24 norm
    values) for SCHED_LEARNED on the current device, with its batch-aware
    slack (None: the library's default)."""
    import numpy as np

    p = np.ascontiguousarray(params, dtype=np.float32)
    k = p.shape[0] if p.ndim == 2 else 1
    nm = np.ascontiguousarray(norm, dtype=np.float32)
    _check(_lib.spmd_model_load(p.ctypes.data, k, nm.ctypes.data, float(sd_threshold)), "spmd_model_load")
    if slack is not None and k:
        _check(_lib.spmd_model_batch_slack(float(slack)), "spmd_model_batch_slack")


def sched_candidates():
    n = int(_lib.spmd_sched_candidates(None, 0))
    arr = (Schedule * n)()
    _lib.spmd_sched_candidates(arr, n)
    return [(s.block, s.items, s.bpf) for s in arr]


def sched_features(kernel_id: int, n: int, ny: int, block_dim: int):
    it = BatchItem(int(kernel_id), int(n), int(ny), int(block_dim), None, None)
    out = (ctypes.c_float * 9)()
    _check(_lib.spmd_sched_features(ctypes.byref(it), out), "spmd_sched_features")
    return list(out)
