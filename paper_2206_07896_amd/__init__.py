"""MI355X (gfx950) SPMD kernel-grid executor -- Python binding.

A thin ctypes layer over ``libspmd.so`` (C ABI in ``include/spmd.h``): it
only marshals arguments (tensor -> device pointer, int -> uint32) and turns
status codes into exceptions.  Every step of every kernel class runs in the
library's HIP kernels; PyTorch provides device memory and streams.

The library must have been built (``python paper_2206_07896_amd/build.py``);
importing this package without it raises ImportError -- there is no
fallback implementation.
"""

from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspmd.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python paper_2206_07896_amd/build.py` "
        "(hipcc, gfx950); this package has no non-HIP implementation")

# torch first: it ships its own HIP runtime under the same soname as the
# system one the library links against, and the process shares whichever
# is loaded first.  Loading torch's first keeps one runtime for both, so
# device pointers and streams from torch are valid in the library.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

SPMD_OK = 0
ERRORS = {
    -1: "INVALID_KERNEL",
    -2: "INVALID_DIM",
    -3: "SHMEM",
    -4: "ARGS",
    -5: "HIP",
    -6: "DEVICE",
    -7: "TIMEOUT",
    -8: "WORKSPACE",
}

REDUCE_I32 = 1
SCAN_I32 = 2
HIST256_U32 = 3
JACOBI5_F32 = 4
GEMM_F32 = 5
WARPTEST = 6
REVERSE_I32 = 7
COMPACT_I32 = 8
JACOBI5T_F32 = 9
NUM_KERNELS = 9
WARPTEST_NCASES = 904
KERNELS = {}


class Dim3(ctypes.Structure):
    _fields_ = [("x", ctypes.c_uint32), ("y", ctypes.c_uint32), ("z", ctypes.c_uint32)]


class SpmdError(RuntimeError):
    def __init__(self, code: int, where: str = ""):
        msg = _lib.spmd_error_string(code).decode()
        if code == -5:
            msg += f" ({_lib.spmd_last_hip_error().decode()})"
        super().__init__(f"{where}: {ERRORS.get(code, code)}: {msg}" if where else msg)
        self.code = code
        self.kind = ERRORS.get(code, str(code))


_P = ctypes.c_void_p
_lib.spmd_launch.argtypes = [ctypes.c_int, Dim3, Dim3, ctypes.c_size_t, ctypes.POINTER(ctypes.c_void_p), _P]
_lib.spmd_launch.restype = ctypes.c_int
_lib.spmd_launch_timed.argtypes = [ctypes.c_int, Dim3, Dim3, ctypes.c_size_t, ctypes.POINTER(ctypes.c_void_p), _P, _P, _P]
_lib.spmd_launch_timed.restype = ctypes.c_int
_lib.spmd_launch_noalloc.argtypes = [ctypes.c_int, Dim3, Dim3, ctypes.c_size_t, ctypes.POINTER(ctypes.c_void_p), _P]
_lib.spmd_launch_noalloc.restype = ctypes.c_int
_lib.spmd_workspace_size.argtypes = [ctypes.c_int, Dim3, Dim3, ctypes.c_uint64]
_lib.spmd_workspace_size.restype = ctypes.c_size_t
_lib.spmd_sync.argtypes = [_P]
_lib.spmd_sync.restype = ctypes.c_int
_lib.spmd_sync_timeout.argtypes = [_P, ctypes.c_uint32]
_lib.spmd_sync_timeout.restype = ctypes.c_int
_lib.spmd_set_spin_limit.argtypes = [ctypes.c_uint32]
_lib.spmd_set_spin_limit.restype = ctypes.c_int
_lib.spmd_kernel_signature.argtypes = [ctypes.c_int]
_lib.spmd_kernel_signature.restype = ctypes.c_char_p
_lib.spmd_kernel_name.argtypes = [ctypes.c_int]
_lib.spmd_kernel_name.restype = ctypes.c_char_p
_lib.spmd_error_string.argtypes = [ctypes.c_int]
_lib.spmd_error_string.restype = ctypes.c_char_p
_lib.spmd_last_hip_error.argtypes = []
_lib.spmd_last_hip_error.restype = ctypes.c_char_p

for _k in range(1, NUM_KERNELS + 1):
    KERNELS[_lib.spmd_kernel_name(_k).decode()] = _k


def lib():
    """The loaded ctypes library (for tests of the C ABI itself)."""
    return _lib


def _dim3(d) -> Dim3:
    if isinstance(d, int):
        return Dim3(d, 1, 1)
    d = tuple(d) + (1,) * (3 - len(d))
    return Dim3(*d)


def _stream_handle(stream) -> int | None:
    if stream is None:
        import torch

        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _ptr(v) -> int:
    if v is None:
        return 0
    if isinstance(v, int):
        return v
    return v.data_ptr()


def _check(rc: int, where: str) -> None:
    if rc != SPMD_OK:
        raise SpmdError(rc, where)


def signature(kernel: int) -> str:
    s = _lib.spmd_kernel_signature(kernel)
    if s is None:
        raise SpmdError(-1, "signature")
    return s.decode()


# classes whose last parameter is a workspace (spmd_launch_noalloc leaves it out)
WORKSPACE_CLASSES = (REDUCE_I32, SCAN_I32, COMPACT_I32)
NOALLOC_REGION_BYTES = (1 << 20) + 16384  # SPMD_NOALLOC_REGION_BYTES


def pack_args(kernel: int, args, sig=None):
    """The host prologue of the paper's parameter packing: one heap object
    per parameter, args[i] pointing at it.  Returns (void** array, keepalive)."""
    sig = signature(kernel) if sig is None else sig
    if len(args) != len(sig):
        raise SpmdError(-4, f"kernel {kernel} takes {len(sig)} arguments, got {len(args)}")
    objs = []
    for kind, v in zip(sig, args):
        if kind == "p":
            objs.append(ctypes.c_void_p(_ptr(v)))
        else:
            objs.append(ctypes.c_uint32(int(v)))
    arr = (ctypes.c_void_p * len(objs))(*[ctypes.cast(ctypes.pointer(o), ctypes.c_void_p) for o in objs])
    return arr, objs


def launch(kernel, grid, block, dyn_shmem: int = 0, args=(), stream=None, events=None) -> None:
    """spmd_launch: enqueue one grid of class ``kernel`` (id or name).  With
    ``events=(start, stop)`` (two :func:`timing_events`), spmd_launch_timed:
    ``start.elapsed_time(stop)`` is then the device time of the launch's
    kernels.  ``start`` may be None: only ``stop`` is bound (free on the
    stream), to be measured from an earlier event."""
    kid = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    arr, keep = pack_args(kid, list(args))
    argv = ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p))
    if events is None:
        rc = _lib.spmd_launch(kid, _dim3(grid), _dim3(block), dyn_shmem, argv, _stream_handle(stream))
        what = "spmd_launch"
    else:
        start, stop = (_event_handle(e) for e in events)
        if stop is None:
            raise ValueError("events=(start, stop): stop must be an event")
        rc = _lib.spmd_launch_timed(kid, _dim3(grid), _dim3(block), dyn_shmem, argv, _stream_handle(stream),
                                    start, stop)
        what = "spmd_launch_timed"
    del keep
    if rc:
        _check(rc, f"{what}({_lib.spmd_kernel_name(kid).decode() if 1 <= kid <= NUM_KERNELS else kid})")


def timing_events(count: int = 2):
    """``count`` torch.cuda.Events with timing enabled whose HIP events
    exist (each recorded once on the current stream), for ``events=`` of
    :func:`launch` and the ops."""
    import torch

    out = []
    for _ in range(count):
        e = torch.cuda.Event(enable_timing=True)
        e.record()
        out.append(e)
    return out


def _event_handle(e) -> int | None:
    if e is None:
        return None
    h = e if isinstance(e, int) else int(e.cuda_event)
    if not h:
        raise ValueError("the event has no HIP event yet: take it from timing_events() or record it once")
    return h


def launch_noalloc(kernel, grid, block, dyn_shmem: int = 0, args=(), stream=None) -> None:
    """spmd_launch_noalloc: as :func:`launch`, with the workspace argument of
    REDUCE_I32, SCAN_I32 and COMPACT_I32 left out (the library's static
    per-device scratch is used instead; nothing is allocated)."""
    kid = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    sig = signature(kid)
    arr, keep = pack_args(kid, list(args), sig[:-1] if kid in WORKSPACE_CLASSES else sig)
    rc = _lib.spmd_launch_noalloc(kid, _dim3(grid), _dim3(block), dyn_shmem,
                                  ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p)), _stream_handle(stream))
    del keep
    _check(rc, f"spmd_launch_noalloc({_lib.spmd_kernel_name(kid).decode() if 1 <= kid <= NUM_KERNELS else kid})")


def workspace_size(kernel, grid, block, n: int) -> int:
    kid = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    return int(_lib.spmd_workspace_size(kid, _dim3(grid), _dim3(block), n))


def sync(stream=None) -> None:
    _check(_lib.spmd_sync(_stream_handle(stream)), "spmd_sync")


def sync_timeout(stream=None, ms: int = 10000) -> None:
    _check(_lib.spmd_sync_timeout(_stream_handle(stream), ms), "spmd_sync_timeout")


def set_spin_limit(polls: int) -> None:
    """Bound on cross-block waits of the current device, in polls (0: the
    default); see spmd_set_spin_limit."""
    _check(_lib.spmd_set_spin_limit(int(polls)), "spmd_set_spin_limit")


from . import ops  # noqa: E402,F401  (tensor-level helpers)
from . import batch  # noqa: E402,F401  (persistent block queue, device inputs)
from . import learned  # noqa: E402,F401  (autotuner and learned cost model)
