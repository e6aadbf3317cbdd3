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

    def __init__(self, items, schedules, workers_per_cu: int = 0, device=None):
        n = len(items)
        if n == 0 or len(schedules) != n:
            raise SpmdError(-4, "Batch: need one schedule per item")
        self._keep = []
        arr = (BatchItem * n)()
        sch = (Schedule * n)()
        for i, (kid, nn, ny, bd, tin, tout) in enumerate(items):
            arr[i] = BatchItem(int(kid), int(nn), int(ny), int(bd), _ptr(tin), _ptr(tout))
            self._keep += [tin, tout]
        for i, (b, it, bpf) in enumerate(schedules):
            sch[i] = Schedule(int(b), int(it), int(bpf))
        size = int(_lib.spmd_batch_workspace_size(arr, sch, n))
        if size == 0:
            raise SpmdError(-2, "spmd_batch_workspace_size (invalid items or schedules)")
        raw = torch.empty(size + 256, dtype=torch.uint8, device=device or "cuda")
        off = (-raw.data_ptr()) % 256
        self.workspace = raw[off:off + size]
        self._raw = raw
        h = _P()
        _check(_lib.spmd_batch_create(arr, sch, n, self.workspace.data_ptr(), size, workers_per_cu, ctypes.byref(h)),
               "spmd_batch_create")
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
