"""The C-ABI library without a GPU: it loads, exports every function the
headers declare, and rejects malformed launches before touching a device."""

import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names.update(re.findall(r"\b(spmd_\w+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def spmd():
    import paper_2206_07896_amd as m

    return m


def test_every_declared_symbol_is_exported(spmd):
    names = declared_functions()
    assert "spmd_launch" in names and "spmd_sync" in names
    lib = ctypes.CDLL(spmd.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_signatures_and_names(spmd):
    assert spmd.signature(spmd.REDUCE_I32) == "pppup"
    assert spmd.signature(spmd.SCAN_I32) == "ppup"
    assert spmd.signature(spmd.HIST256_U32) == "ppu"
    assert spmd.signature(spmd.JACOBI5_F32) == "ppuu"
    assert spmd.signature(spmd.GEMM_F32) == "pppuuu"
    assert spmd.signature(spmd.WARPTEST) == "ppp"
    assert spmd.signature(spmd.REVERSE_I32) == "pu"
    assert set(spmd.KERNELS) == {"reduce_i32", "scan_i32", "hist256_u32", "jacobi5_f32", "gemm_f32", "warptest",
                                 "reverse_i32"}
    lib = spmd.lib()
    assert lib.spmd_kernel_signature(0) is None
    assert lib.spmd_kernel_signature(spmd.NUM_KERNELS + 1) is None


def test_error_strings(spmd):
    for code in [0, -1, -2, -3, -4, -5, -6, -7, -8]:
        assert spmd.lib().spmd_error_string(code)
    assert spmd.lib().spmd_error_string(-99) == b"unknown status"


def test_workspace_sizes(spmd):
    assert spmd.workspace_size(spmd.REDUCE_I32, 4096, 256, 1 << 20) == 16
    assert spmd.workspace_size(spmd.SCAN_I32, 8192, 512, 1 << 26) == 16 + 8 * 8192
    assert spmd.workspace_size(spmd.HIST256_U32, 10, 256, 100) == 0
    assert spmd.workspace_size(99, 1, 1, 1) == 0


def _raw_launch(spmd, kid, grid, block, shm, args):
    if args is None:
        argp = None
    else:
        arr, keep = spmd.pack_args(kid, args) if kid in range(1, spmd.NUM_KERNELS + 1) else (None, None)
        argp = ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p)) if arr is not None else None
    return spmd.lib().spmd_launch(kid, spmd._dim3(grid), spmd._dim3(block), shm, argp, None)


@pytest.mark.parametrize("kid", [0, -3, 8, 1000])
def test_unknown_kernel(spmd, kid):
    assert _raw_launch(spmd, kid, 1, 64, 0, None) == -1


@pytest.mark.parametrize("grid,block", [((0, 1, 1), 64), ((1, 0, 1), 64), (1, (64, 1, 0)), (1, (0, 1, 1)),
                                        (1, 2048), (1, (32, 33, 1)), ((1 << 16, 1 << 16, 1), 64)])
def test_bad_dimensions(spmd, grid, block):
    assert _raw_launch(spmd, spmd.REDUCE_I32, grid, block, 0, [0, 0, 0, 1, 0]) == -2


def test_null_args(spmd):
    assert _raw_launch(spmd, spmd.REDUCE_I32, 1, 64, 0, None) == -4
    lib = spmd.lib()
    arr = (ctypes.c_void_p * 5)()
    rc = lib.spmd_launch(spmd.REDUCE_I32, spmd._dim3(1), spmd._dim3(64), 0,
                         ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p)), None)
    assert rc == -4


def test_binding_arity_check(spmd):
    with pytest.raises(spmd.SpmdError) as e:
        spmd.pack_args(spmd.SCAN_I32, [0, 0])
    assert e.value.kind == "ARGS"
