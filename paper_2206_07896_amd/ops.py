"""Tensor-level helpers over :func:`launch`: allocate outputs and workspace
with PyTorch, pick the launch shape, enqueue.  They do no arithmetic of
their own.  All tensors must live on the current HIP device; int32 tensors
carry uint32 data bit for bit (keys, histogram counts).  The single-launch
helpers take ``events=(start, stop)`` (from :func:`timing_events`) to time
their launch's kernels on the device (spmd_launch_timed).
"""

from __future__ import annotations

import torch

from . import (COMPACT_I32, GEMM_F32, HIST256_U32, JACOBI5_F32, JACOBI5T_F32, REDUCE_I32, REVERSE_I32, SCAN_I32,
               WARPTEST, WARPTEST_NCASES, launch, workspace_size)


def _cdiv(a: int, b: int) -> int:
    return -(-a // b)


def _check_dev(*ts):
    for t in ts:
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError("tensors must be contiguous and on the GPU")


def workspace(kernel, grid, block, n: int, device=None) -> torch.Tensor:
    """A zero-filled workspace for ``kernel`` (reusable across launches on
    one stream)."""
    nbytes = max(16, workspace_size(kernel, grid, block, n))
    return torch.zeros(_cdiv(nbytes, 16) * 16, dtype=torch.uint8, device=device or "cuda")


def reduce_i32(x: torch.Tensor, grid: int = 4096, block: int = 256, partials=None, out=None, ws=None,
               dyn_shmem: int | None = None, stream=None, events=None):
    _check_dev(x)
    n = x.numel()
    if partials is None:
        partials = torch.empty(grid, dtype=torch.int32, device=x.device)
    if out is None:
        out = torch.empty(1, dtype=torch.int32, device=x.device)
    if ws is None:
        ws = workspace(REDUCE_I32, grid, block, n, x.device)
    shm = 4 * block if dyn_shmem is None else dyn_shmem
    launch(REDUCE_I32, grid, block, shm, [x, partials, out, n, ws], stream, events)
    return partials, out


def scan_grid(n: int, block: int = 512, items: int = 16) -> int:
    return max(1, _cdiv(n, block * items))


def scan_i32(x: torch.Tensor, block: int = 512, items: int = 16, y=None, ws=None, stream=None, events=None):
    _check_dev(x)
    n = x.numel()
    grid = scan_grid(n, block, items)
    if y is None:
        y = torch.empty_like(x)
    if ws is None:
        ws = workspace(SCAN_I32, grid, block, n, x.device)
    launch(SCAN_I32, grid, block, 0, [x, y, n, ws], stream, events)
    return y


def compact_grid(n: int, block: int = 256, items: int = 16) -> int:
    return max(1, _cdiv(n, block * items))


def compact_i32(x: torch.Tensor, t: int, block: int = 256, items: int = 16, y=None, count=None, ws=None,
                stream=None, events=None):
    """Elements of x greater than t, in order: returns (y, count); y[:count]
    holds them."""
    _check_dev(x)
    n = x.numel()
    grid = compact_grid(n, block, items)
    if y is None:
        y = torch.empty_like(x)
    if count is None:
        count = torch.zeros(1, dtype=torch.int32, device=x.device)
    if ws is None:
        ws = workspace(COMPACT_I32, grid, block, n, x.device)
    launch(COMPACT_I32, grid, block, 0, [x, y, count, n, int(t) & 0xFFFFFFFF, ws], stream, events)
    return y, count


def hist256_u32(keys: torch.Tensor, grid: int = 256, block: int = 1024, hist=None, stream=None, events=None):
    _check_dev(keys)
    if hist is None:
        hist = torch.empty(256, dtype=torch.int32, device=keys.device)
    launch(HIST256_U32, grid, block, 0, [keys, hist, keys.numel()], stream, events)
    return hist


def jacobi_grid(nx: int, ny: int, block=(16, 16), cells: int = 1):
    bx, by = block
    return (_cdiv(nx, bx), _cdiv(ny, by * cells))


def jacobi5_f32(u: torch.Tensor, out=None, block=(16, 16), cells: int = 1, stream=None, events=None):
    _check_dev(u)
    ny, nx = u.shape
    if out is None:
        out = torch.empty_like(u)
    launch(JACOBI5_F32, jacobi_grid(nx, ny, block, cells), (block[0], block[1], 1), 0, [u, out, nx, ny], stream, events)
    return out


def jacobi5_sweeps(u: torch.Tensor, sweeps: int, block=(16, 16), cells: int = 1, scratch=None, stream=None):
    """``sweeps`` launches ping-ponging between u (left untouched) and two
    buffers; returns the buffer holding the result."""
    a = u.clone() if sweeps else u
    b = torch.empty_like(u) if scratch is None else scratch
    src, dst = a, b
    for _ in range(sweeps):
        jacobi5_f32(src, dst, block, cells, stream)
        src, dst = dst, src
    return src


def jacobi5t_grid(nx: int, ny: int, sweeps: int):
    """Grid of the fused-sweep class: (256 - 2H) x 64 interior tiles, halo
    H = 4 for up to 4 sweeps, else 8."""
    h = 4 if sweeps <= 4 else 8
    return (_cdiv(nx, 256 - 2 * h), _cdiv(ny, 64))


def jacobi5t_f32(u: torch.Tensor, sweeps: int, out=None, stream=None, events=None):
    """``sweeps`` (1..8) sweeps in one launch (SPMD_JACOBI5T_F32)."""
    _check_dev(u)
    ny, nx = u.shape
    if out is None:
        out = torch.empty_like(u)
    launch(JACOBI5T_F32, jacobi5t_grid(nx, ny, sweeps), (256, 1, 1), 0, [u, out, nx, ny, sweeps], stream, events)
    return out


def jacobi5t_sweeps(u: torch.Tensor, sweeps: int, per_launch: int = 4, scratch=None, stream=None):
    """``sweeps`` sweeps as launches of up to ``per_launch`` fused sweeps,
    ping-ponging between a copy of u and a second buffer."""
    a = u.clone() if sweeps else u
    b = torch.empty_like(u) if scratch is None else scratch
    src, dst = a, b
    left = sweeps
    while left:
        k = min(per_launch, left)
        jacobi5t_f32(src, k, dst, stream)
        src, dst = dst, src
        left -= k
    return src


def gemm_f32(A: torch.Tensor, B: torch.Tensor, C=None, tile: int = 128, stream=None, events=None):
    _check_dev(A, B)
    M, K = A.shape
    K2, N = B.shape
    assert K == K2
    if C is None:
        C = torch.empty((M, N), dtype=torch.float32, device=A.device)
    launch(GEMM_F32, (_cdiv(N, tile), _cdiv(M, tile)), 256, 0, [A, B, C, M, N, K], stream, events)
    return C


def warptest(val: torch.Tensor, pred: torch.Tensor, grid: int, block: int, out=None, stream=None):
    _check_dev(val, pred)
    total = grid * block
    if out is None:
        out = torch.empty((WARPTEST_NCASES, total), dtype=torch.int32, device=val.device)
    launch(WARPTEST, grid, block, 0, [val, pred, out], stream)
    return out


def reverse_i32(d: torch.Tensor, stream=None):
    _check_dev(d)
    n = d.numel()
    launch(REVERSE_I32, 1, n, 4 * n, [d, n], stream)
    return d
