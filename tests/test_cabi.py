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
    assert spmd.workspace_size(spmd.REDUCE_I32, 4096, 256, 1 << 20) == 65 * 128 + 8 * 4096
    assert spmd.workspace_size(spmd.SCAN_I32, 8192, 512, 1 << 26) == 256 + 8 * 8192
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


# --------------------------------------------------------------------------
# batch ABI (host-side parts)
# --------------------------------------------------------------------------

def test_batch_item_blocks(spmd):
    ib = spmd.batch.item_blocks
    R, S, H, J = spmd.REDUCE_I32, spmd.SCAN_I32, spmd.HIST256_U32, spmd.JACOBI5_F32
    assert ib(R, 1000, 1, 64, 4) == 4          # ceil(1000 / 256)
    assert ib(R, 0, 1, 64, 4) == 1             # an empty reduction still writes its total
    assert ib(S, 1 << 20, 1, 512, 16) == 128
    assert ib(H, (1 << 20) + 1, 1, 256, 16) == 257
    assert ib(J, 100, 50, 256, 2) == 2 * 7     # 64-wide blocks of 4 rows x 2 cells
    assert ib(J, 8192, 8192, 512, 8) == 128 * 128
    for bad in [(S, 100, 1, 96, 4), (S, 100, 1, 1024, 4), (R, 100, 1, 64, 3), (J, 100, 1, 64, 16), (J, 0, 5, 64, 1),
                (6, 100, 1, 64, 1)]:
        assert ib(*bad) == 0, bad
    assert ib(R, 100, 1, 64, 1, bpf=0) == 0


def _items(spmd, specs):
    import ctypes

    B = spmd.batch
    arr = (B.BatchItem * len(specs))()
    sch = (B.Schedule * len(specs))()
    for i, (kid, n, ny, s) in enumerate(specs):
        arr[i] = B.BatchItem(kid, n, ny, 64, 0x1000, 0x2000)
        sch[i] = B.Schedule(*s)
    return arr, sch


def test_batch_workspace_and_validation(spmd):
    import ctypes

    lib = spmd.lib()
    R, S, H, J = spmd.REDUCE_I32, spmd.SCAN_I32, spmd.HIST256_U32, spmd.JACOBI5_F32
    arr, sch = _items(spmd, [(R, 1000, 1, (64, 4, 1)), (S, 5000, 1, (128, 2, 3)), (H, 10, 1, (512, 16, 1)),
                             (J, 30, 20, (256, 2, 2))])
    size = lib.spmd_batch_workspace_size(arr, sch, 4)
    # run area (cursors + reduce ticket/status + scan status) + baseline scratch + 4 descriptors + maps
    assert size >= 256 + (65 * 128 + 8 * 4) + 8 * 20 + 4 * 64 and size % 256 == 0
    h = ctypes.c_void_p()
    # workspace checks come before any device work
    assert lib.spmd_batch_create(arr, sch, 4, None, size, 0, ctypes.byref(h)) == -8
    assert lib.spmd_batch_create(arr, sch, 4, 0x1000 + 16, size, 0, ctypes.byref(h)) == -8
    assert lib.spmd_batch_create(arr, sch, 4, 0x100000, size - 1, 0, ctypes.byref(h)) == -8
    bad_k, bad_s = _items(spmd, [(spmd.GEMM_F32, 10, 1, (64, 1, 1))])
    assert lib.spmd_batch_workspace_size(bad_k, bad_s, 1) == 0
    assert lib.spmd_batch_create(bad_k, bad_s, 1, 0x100000, 1 << 20, 0, ctypes.byref(h)) == -1
    bad_k, bad_s = _items(spmd, [(S, 10, 1, (96, 1, 1))])
    assert lib.spmd_batch_create(bad_k, bad_s, 1, 0x100000, 1 << 20, 0, ctypes.byref(h)) == -2
    assert lib.spmd_batch_create(arr, sch, 0, 0x100000, 1 << 20, 0, ctypes.byref(h)) == -4
    assert lib.spmd_batch_launch(None, None) == -4
    assert lib.spmd_batch_destroy(None) == -4
