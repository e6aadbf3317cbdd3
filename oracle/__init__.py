"""CPU oracle for SPMD kernel-grid execution.  TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
use this package.  The product path (the HIP library and its binding) never
imports, links or calls anything here, and this package never imports the
product path: the two share only the seeded input generators in ``synth``.

What it computes (C sources in this directory):

* ``mpmd.c`` -- the executor.  A block body runs the way the paper's
  SPMD-to-MPMD transformation leaves it (Section III-B3): one thread loop per
  barrier-delimited region, and nested warp/lane loops split at each warp
  operation; shared memory is a per-block poisoned array, global memory is
  bounds-checked host arrays (Section III-B1); blockIdx/blockDim/dynamic
  shared memory are set per block at run time (Section III-B2, Section IV
  "Execute fetched kernel").  Blocks run serially or on a thread pool with a
  mutex-guarded task queue and coarse-grained fetching (Section IV,
  Section IV-A).
* ``classes.c`` -- the kernel classes as MPMD block bodies: block tree
  reduction, warp-shuffle scan, LDS sub-histogram, 5-point Jacobi sweep,
  tiled GEMM, 32-lane warp-operation conformance, and the paper's
  dynamic-shared-memory reversal example (Section III, listing
  ``cuda_reverse``).
* ``fp64.c`` -- FP64 Jacobi and GEMM by their plain definitions, and a fast
  whole-grid fp32 Jacobi with the class's association.

Every function raises :class:`OracleError` on a launch the executor refuses
or on a detected race (shared-memory read before write, divergent barrier,
out-of-bounds access).
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["mpmd.c", "classes.c", "fp64.c", "select.c"]
_lock = threading.Lock()
_lib = None

OX_ERRORS = {
    -1: "BOUNDS",
    -2: "UNINIT",
    -3: "DIVERGENT",
    -4: "CONFIG",
    -5: "NOMEM",
}


class OracleError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"oracle error {OX_ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.kind = OX_ERRORS.get(code, str(code))


def build(force: bool = False) -> str:
    """Compile the oracle's C sources into ``liboracle.so`` with gcc."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES]
    if not force and os.path.exists(_SO):
        so_t = os.path.getmtime(_SO)
        if all(os.path.getmtime(s) <= so_t for s in srcs + [os.path.join(_HERE, "mpmd.h")]):
            return _SO
    tmp = _SO + f".tmp{os.getpid()}"
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-strict-aliasing",
           "-fopenmp", "-pthread", "-shared", "-fPIC", "-Wall", "-o", tmp] + srcs
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_SO)
            P = ctypes.c_void_p
            U32, U64, I32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
            C = ctypes.c_char_p
            sig = {
                "oracle_reduce_i32": [P, U32, U32, U32, P, P, U64, I32, U32, I32, C],
                "oracle_scan_i32": [P, U32, U32, U32, P, U64, I32, C],
                "oracle_hist256_u32": [P, U32, U32, U32, P, U64, I32, U32, C],
                "oracle_jacobi5_f32": [P, P, U32, U32, U32, U32, U64, I32, C],
                "oracle_gemm_f32": [P, P, P, U32, U32, U32, U64, I32, C],
                "oracle_warptest": [P, P, U32, U32, P, U64, C],
                "oracle_reverse_i32": [P, U32, U64, I32, C],
                "oracle_pool_probe": [U32, I32, U32, P, P, P, C],
                "oracle_jacobi5_f64": [P, U32, U32, U32, P],
                "oracle_jacobi5_f32_sweeps": [P, U32, U32, U32, P],
                "oracle_gemm_f64": [P, P, U32, U32, U32, P],
                "oracle_gemm_f64_entries": [P, P, U32, U32, P, P, U64, P],
                "oracle_compact_i32": [P, U64, ctypes.c_int32, P, P],
            }
            for name, args in sig.items():
                f = getattr(lib, name)
                f.argtypes = args
                f.restype = ctypes.c_int
            lib.oracle_warptest_ncases.restype = ctypes.c_uint32
            lib.oracle_gemm_f64.restype = None
            lib.oracle_gemm_f64_entries.restype = None
            lib.oracle_pool_shutdown.restype = None
            _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc: int, msg) -> None:
    if rc != 0:
        raise OracleError(rc, msg.value.decode(errors="replace"))


def _c(a, dtype) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=dtype)


# ---------------------------------------------------------------------------
# kernel classes (block executor)
# ---------------------------------------------------------------------------

def reduce_i32(x, grid: int, block: int, order_seed: int = 0, pool: int = 0, bpf: int = 0,
               skip_barrier: bool = False):
    """Block tree reduction with one partial per block; the last block to
    finish sums the partials.  Block b owns x[b*S : (b+1)*S] with
    S = 4 * ceil(n / (4 * grid)).  Returns (partials[grid], total) as int32,
    sums taken modulo 2^32."""
    lib = _load()
    x = _c(x, np.int32)
    partials = np.zeros(grid, np.int32)
    out = np.zeros(1, np.int32)
    msg = ctypes.create_string_buffer(256)
    rc = lib.oracle_reduce_i32(_p(x), x.size, grid, block, _p(partials), _p(out), order_seed, pool, bpf,
                               int(skip_barrier), msg)
    _check(rc, msg)
    return partials, int(out[0])


def scan_i32(x, block: int = 512, items: int = 16, order_seed: int = 0, pool: int = 0) -> np.ndarray:
    """Inclusive prefix sum modulo 2^32 (int32 view), tiles of block*items
    elements: thread-serial scan, 32-lane shfl_up warp scan, warp totals
    through shared memory, then the grid carry (three launches)."""
    lib = _load()
    x = _c(x, np.int32)
    y = np.zeros(x.size, np.int32)
    msg = ctypes.create_string_buffer(256)
    rc = lib.oracle_scan_i32(_p(x), x.size, block, items, _p(y), order_seed, pool, msg)
    _check(rc, msg)
    return y


def hist256_u32(keys, grid: int, block: int, order_seed: int = 0, pool: int = 0, bpf: int = 0) -> np.ndarray:
    """256-bin histogram of keys & 255: per-block shared sub-histogram with
    shared atomics, then global atomics for the non-zero bins."""
    lib = _load()
    keys = _c(keys, np.uint32)
    hist = np.zeros(256, np.uint32)
    msg = ctypes.create_string_buffer(256)
    rc = lib.oracle_hist256_u32(_p(keys), keys.size, grid, block, _p(hist), order_seed, pool, bpf, msg)
    _check(rc, msg)
    return hist


def jacobi5_f32(u, bx: int = 16, by: int = 16, order_seed: int = 0, pool: int = 0) -> np.ndarray:
    """One Jacobi sweep of a 2-D fp32 grid (ny rows of nx) by the block
    executor: a bx x by block stages its tile and a one-cell halo in shared
    memory, barrier, then computes.  Border cells are copied."""
    lib = _load()
    u = _c(u, np.float32)
    ny, nx = u.shape
    out = np.zeros_like(u)
    msg = ctypes.create_string_buffer(256)
    rc = lib.oracle_jacobi5_f32(_p(u), _p(out), nx, ny, bx, by, order_seed, pool, msg)
    _check(rc, msg)
    return out


def jacobi5_f32_sweeps(u, sweeps: int) -> np.ndarray:
    """``sweeps`` fp32 Jacobi sweeps by a whole-grid loop, same association
    as the class: 0.25f * ((N + S) + (W + E))."""
    lib = _load()
    u = _c(u, np.float32)
    ny, nx = u.shape
    out = np.zeros_like(u)
    rc = lib.oracle_jacobi5_f32_sweeps(_p(u), nx, ny, sweeps, _p(out))
    if rc:
        raise OracleError(rc, "jacobi f32 sweeps")
    return out


def jacobi5_f64(u, sweeps: int) -> np.ndarray:
    """``sweeps`` Jacobi sweeps in double from fp32 initial values."""
    lib = _load()
    u = _c(u, np.float32)
    ny, nx = u.shape
    out = np.zeros((ny, nx), np.float64)
    rc = lib.oracle_jacobi5_f64(_p(u), nx, ny, sweeps, _p(out))
    if rc:
        raise OracleError(rc, "jacobi f64")
    return out


def gemm_f32(A, B, order_seed: int = 0, pool: int = 0) -> np.ndarray:
    """C = A @ B (row-major fp32) by the block executor: 64x64 output tile
    per block of 256 threads, 16-deep k-tiles staged in shared memory, fp32
    accumulation in ascending k."""
    lib = _load()
    A = _c(A, np.float32)
    B = _c(B, np.float32)
    M, K = A.shape
    K2, N = B.shape
    assert K == K2
    C = np.zeros((M, N), np.float32)
    msg = ctypes.create_string_buffer(256)
    rc = lib.oracle_gemm_f32(_p(A), _p(B), _p(C), M, N, K, order_seed, pool, msg)
    _check(rc, msg)
    return C


def gemm_f64(A, B) -> np.ndarray:
    """C = A @ B in double, k ascending (plain triple loop)."""
    lib = _load()
    A = _c(A, np.float32)
    B = _c(B, np.float32)
    M, K = A.shape
    N = B.shape[1]
    C = np.zeros((M, N), np.float64)
    lib.oracle_gemm_f64(_p(A), _p(B), M, N, K, _p(C))
    return C


def gemm_f64_entries(A, B, ii, jj) -> np.ndarray:
    """Selected entries C[ii[t], jj[t]] of A @ B in double."""
    lib = _load()
    A = _c(A, np.float32)
    B = _c(B, np.float32)
    K = A.shape[1]
    N = B.shape[1]
    ii = _c(ii, np.uint32)
    jj = _c(jj, np.uint32)
    out = np.zeros(ii.size, np.float64)
    lib.oracle_gemm_f64_entries(_p(A), _p(B), N, K, _p(ii), _p(jj), ii.size, _p(out))
    return out


def compact_i32(x, t: int):
    """The elements of x greater than t, in order (select.c)."""
    lib = _load()
    x = _c(x, np.int32)
    y = np.empty(max(1, x.size), np.int32)
    m = ctypes.c_uint64(0)
    lib.oracle_compact_i32(_p(x), x.size, int(t), _p(y), ctypes.byref(m))
    return y[: m.value].copy()


WARPTEST_NCASES = None


def warptest_ncases() -> int:
    return int(_load().oracle_warptest_ncases())


def warptest_case(c: int):
    """Decode conformance case c into (op, param, width) or a vote case.

    c in [0, 768): op in (shfl, up, down, xor) = c // 192, width 1 << ((c//32) % 6),
    parameter c % 32.  c in [768, 864): vote in (ballot, any, all) =
    (c-768)//32 over predicate bit (c-768) % 32.  c in [864, 904): the
    constant-parameter forms, op (up, down, xor, shfl) = k // 10, width
    32 >> ((k//5) % 2), parameter 1 << (k % 5) with k = c - 864."""
    if c < 768:
        return ("shfl", "up", "down", "xor")[c // 192], c % 32, 1 << ((c // 32) % 6)
    if c < 864:
        return ("ballot", "any", "all")[(c - 768) // 32], (c - 768) % 32, 32
    k = c - 864
    return ("up", "down", "xor", "shfl")[k // 10], 1 << (k % 5), 32 >> ((k // 5) % 2)


def warptest(val, pred, grid: int, block: int, order_seed: int = 0) -> np.ndarray:
    """Every 32-lane warp operation case on every thread: out[c, gtid]."""
    lib = _load()
    val = _c(val, np.int32)
    pred = _c(pred, np.uint32)
    nc = warptest_ncases()
    total = grid * block
    assert val.size == total and pred.size == total
    out = np.zeros((nc, total), np.int32)
    msg = ctypes.create_string_buffer(256)
    rc = lib.oracle_warptest(_p(val), _p(pred), grid, block, _p(out), order_seed, msg)
    _check(rc, msg)
    return out


def reverse_i32(d, order_seed: int = 0, skip_barrier: bool = False) -> np.ndarray:
    """The paper's dynamicReverse: one block of n threads, n*4 bytes of
    dynamic shared memory, s[t] = d[t]; barrier; d[t] = s[n-t-1].
    ``skip_barrier`` runs both statements in one thread loop (a planted
    race that the poisoned shared memory must catch)."""
    lib = _load()
    d = _c(d, np.int32).copy()
    msg = ctypes.create_string_buffer(256)
    rc = lib.oracle_reverse_i32(_p(d), d.size, order_seed, int(skip_barrier), msg)
    _check(rc, msg)
    return d


def pool_probe(grid: int, pool: int, bpf: int = 0):
    """Run an empty grid on the thread-pool runtime; return
    (atomic fetches, workers that executed blocks, blocks per fetch used)."""
    lib = _load()
    f = np.zeros(1, np.uint64)
    w = np.zeros(1, np.uint32)
    b = np.zeros(1, np.uint32)
    msg = ctypes.create_string_buffer(256)
    rc = lib.oracle_pool_probe(grid, pool, bpf, _p(f), _p(w), _p(b), msg)
    _check(rc, msg)
    return int(f[0]), int(w[0]), int(b[0])


def pool_shutdown() -> None:
    _load().oracle_pool_shutdown()
