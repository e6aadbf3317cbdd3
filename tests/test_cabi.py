"""The C-ABI library without a GPU: it loads, exports every function the
headers declare, and rejects malformed launches before touching a device."""

import ctypes
import glob
import os
import re

import numpy as np
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
    assert spmd.signature(spmd.COMPACT_I32) == "pppuup"
    assert spmd.signature(spmd.JACOBI5T_F32) == "ppuuu"
    assert set(spmd.KERNELS) == {"reduce_i32", "scan_i32", "hist256_u32", "jacobi5_f32", "gemm_f32", "warptest",
                                 "reverse_i32", "compact_i32", "jacobi5t_f32"}
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


@pytest.mark.parametrize("kid", [0, -3, 10, 1000])
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


def test_launch_timed_validation(spmd):
    """spmd_launch_timed refuses a null stop event before any device call, and
    passes spmd_launch's own refusals through without touching the events
    (here stand-in handles that are never dereferenced)."""
    lib = spmd.lib()
    arr = (ctypes.c_void_p * 5)()
    argp = ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p))
    d1, d64 = spmd._dim3(1), spmd._dim3(64)
    assert lib.spmd_launch_timed(spmd.REDUCE_I32, d1, d64, 0, argp, None, None, None) == -4
    assert lib.spmd_launch_timed(spmd.REDUCE_I32, d1, d64, 0, argp, None, 16, None) == -4
    assert lib.spmd_launch_timed(99, d1, d64, 0, argp, None, None, 32) == -1  # a null start event is allowed
    assert lib.spmd_launch_timed(99, d1, d64, 0, argp, None, 16, 32) == -1
    assert lib.spmd_launch_timed(spmd.REDUCE_I32, spmd._dim3((0, 1, 1)), d64, 0, argp, None, 16, 32) == -2
    assert lib.spmd_launch_timed(spmd.REDUCE_I32, d1, d64, 0, argp, None, 16, 32) == -4  # null arguments


def _raw_noalloc(spmd, kid, grid, block, args):
    argp = None
    if args is not None:
        sig = spmd.signature(kid)
        arr, keep = spmd.pack_args(kid, args, sig[:-1] if kid in spmd.WORKSPACE_CLASSES else sig)
        argp = ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p))
    return spmd.lib().spmd_launch_noalloc(kid, spmd._dim3(grid), spmd._dim3(block), 0, argp, None)


def test_noalloc_validation(spmd):
    """spmd_launch_noalloc refuses, before touching a device: an unknown
    class, missing arguments, a zero dimension, and a grid whose workspace
    does not fit the static region (any grid of up to 2^17 blocks fits)."""
    lib = spmd.lib()
    assert lib.spmd_launch_noalloc(99, spmd._dim3(1), spmd._dim3(64), 0, None, None) == -1
    for kid in spmd.WORKSPACE_CLASSES:
        assert lib.spmd_launch_noalloc(kid, spmd._dim3(1), spmd._dim3(64), 0, None, None) == -4
        args = [16] * (len(spmd.signature(kid)) - 1)  # never dereferenced: every case is refused
        assert _raw_noalloc(spmd, kid, (0, 1, 1), 64, args) == -2
        fits = 1 << 17
        assert spmd.workspace_size(kid, fits, 64, 0) <= spmd.NOALLOC_REGION_BYTES
        over = fits
        while spmd.workspace_size(kid, over, 64, 0) <= spmd.NOALLOC_REGION_BYTES:
            over += 1
        assert _raw_noalloc(spmd, kid, over, 64, args) == -8
    # a class without a workspace is validated as by spmd_launch
    assert _raw_noalloc(spmd, spmd.HIST256_U32, 1, 2048, [16, 16, 16]) == -2


def test_model_batch_slack_validation(spmd):
    """A negative or non-finite slack is refused before any device call."""
    lib = spmd.batch._lib
    for bad in (-1.0, float("nan"), float("inf")):
        assert lib.spmd_model_batch_slack(bad) == -4


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
    assert ib(R, 100, 1, 64, 1, bpf=0) == 2   # bpf 0 (own grid): same logical blocks


def _items(spmd, specs):
    import ctypes

    B = spmd.batch
    arr = (B.BatchItem * len(specs))()
    sch = (B.Schedule * len(specs))()
    for i, (kid, n, ny, s) in enumerate(specs):
        arr[i] = B.BatchItem(kid, n, ny, 64, (1 << 32) + (i << 28), (1 << 36) + (i << 28))  # disjoint buffers
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


def test_schedule_candidates_table(spmd):
    from paper_2206_07896_amd import batch as B

    c = B.sched_candidates()
    assert len(c) == 144 and len(set(c)) == 144
    assert c[0] == (64, 1, 1) and c[-1] == (512, 32, 32)
    assert sorted(c) == c  # block, then items, then bpf ascending
    assert {b for b, _, _ in c} == {64, 128, 256, 512}
    assert {i for _, i, _ in c} == {1, 2, 4, 8, 16, 32}
    assert {f for _, _, f in c} == {1, 2, 4, 8, 16, 32}


def test_candidate_validity_matches_library(spmd):
    """The binding's per-class candidate mask (what the tuner sweeps and
    the cost model may choose) is exactly the set of candidates the
    library's chunk table accepts: Jacobi at most 8 items, 32 items for
    scan only."""
    from paper_2206_07896_amd import learned as L

    for kid in (spmd.REDUCE_I32, spmd.SCAN_I32, spmd.HIST256_U32, spmd.JACOBI5_F32):
        nx, ny = (300, 200) if kid == spmd.JACOBI5_F32 else (100000, 1)
        ch = L.sched_chunks([{"kid": kid, "nx": nx, "ny": ny, "block_dim": 256}])[0]
        lib_ok = ch != 0xFFFFFFFF
        assert np.array_equal(L.valid_candidates(kid), lib_ok), kid
    items = np.array([it for _, it, _ in L.CANDIDATES])
    assert not L.valid_candidates(spmd.JACOBI5_F32)[items > 8].any()
    assert L.valid_candidates(spmd.SCAN_I32)[items == 32].all()
    assert not L.valid_candidates(spmd.REDUCE_I32)[items == 32].any()


def test_launch_features_closed_forms(spmd):
    from paper_2206_07896_amd import batch as B

    # REDUCE at blockDim 256: 1 KiB of shared memory, 8 tree levels + the load barrier
    f = B.sched_features(spmd.REDUCE_I32, 1 << 20, 1, 256)
    assert f == [1.0, 0.0, 0.0, 0.0, 20.0, 8.0, 10.0, 9.0, 0.0]
    # SCAN at blockDim 512: 16 warp totals + the carry, two barriers, 2 x 5 shuffles
    f = B.sched_features(spmd.SCAN_I32, 1 << 26, 1, 512)
    assert f[:6] == [0.0, 1.0, 0.0, 0.0, 26.0, 9.0] and f[7:] == [2.0, 10.0]
    assert abs(f[6] - np.log2(4 * 16 + 4)) < 1e-6
    # JACOBI counts nx * ny elements
    f = B.sched_features(spmd.JACOBI5_F32, 64, 32, 128)
    assert f[3] == 1.0 and f[4] == 11.0 and f[5] == 7.0
    # HIST, and n = 0 is treated as one element
    f = B.sched_features(spmd.HIST256_U32, 0, 1, 64)
    assert f[2] == 1.0 and f[4] == 0.0 and f[6] == 10.0


def test_launch_batch_rejects_unbatchable_launches(spmd):
    """Descriptor validation needs no device: the workspace query returns 0
    for launches that cannot be batched."""
    import ctypes as C

    from paper_2206_07896_amd import batch as B

    def desc(kid, grid, block, args):
        arr = (C.c_void_p * len(args))(*args)
        return B.LaunchDesc(kid, (C.c_uint32 * 3)(*grid), (C.c_uint32 * 3)(*block), 0,
                            C.cast(arr, C.POINTER(C.c_void_p))), arr

    n = C.c_uint32(1000)
    p, q = C.c_void_p(0x100000), C.c_void_p(0x200000)  # keys, bins: disjoint
    ptrs = [C.cast(C.pointer(p), C.c_void_p).value, C.cast(C.pointer(q), C.c_void_p).value,
            C.cast(C.pointer(q), C.c_void_p).value, C.cast(C.pointer(n), C.c_void_p).value]
    ok, keep = desc(spmd.HIST256_U32, (4, 1, 1), (256, 1, 1), ptrs[:2] + [ptrs[3]])
    lib = spmd.lib()
    one = (B.LaunchDesc * 1)(ok)
    assert lib.spmd_launch_batch_workspace_size(one, 1) > 0
    for kid, grid, block in ((spmd.GEMM_F32, (4, 1, 1), (256, 1, 1)),       # not a batchable class
                             (spmd.HIST256_U32, (0, 1, 1), (256, 1, 1)),    # empty grid
                             (spmd.HIST256_U32, (4, 1, 1), (2048, 1, 1))):  # block over 1024
        bad, keep2 = desc(kid, grid, block, ptrs[:2] + [ptrs[3]])
        assert lib.spmd_launch_batch_workspace_size((B.LaunchDesc * 1)(bad), 1) == 0
    assert lib.spmd_launch_batch_workspace_size(one, 0) == 0
    # learned mode without a model, bad mode, missing workspace: errors, no device work
    assert lib.spmd_launch_batch(one, 1, 7, None, 0, None) == -4
    assert lib.spmd_launch_batch(one, 1, 0, None, 0, None) == -8


def test_launch_batch_workspace_covers_every_schedule(spmd):
    """The bound spmd_launch_batch reserves must hold the plan of any
    schedule the cost model may pick: for a seeded mix of launches and for
    every candidate applied to all of them, the plan fits."""
    import ctypes as C

    from paper_2206_07896_amd import batch as B

    rng = np.random.default_rng(3)
    cands = B.sched_candidates()
    keep = []
    descs, items = [], []
    for i in range(24):
        kid = [spmd.REDUCE_I32, spmd.SCAN_I32, spmd.HIST256_U32, spmd.JACOBI5_F32][i % 4]
        n = int(rng.integers(1, 1 << 20))
        bd = int(rng.choice([32, 64, 96, 128, 256, 512, 1024]))
        vals = [C.c_void_p((i + 1) << 32), C.c_void_p(((i + 1) << 32) + (1 << 28))]  # input, output: disjoint
        if kid == spmd.JACOBI5_F32:
            nx = ny = max(1, int(np.sqrt(n)))
            ints = [C.c_uint32(nx), C.c_uint32(ny)]
            args = vals + ints
            items.append(B.BatchItem(kid, nx, ny, bd, vals[0].value, vals[1].value))
        else:
            ints = [C.c_uint32(n)]
            args = (vals[:1] + [vals[1], vals[1]] + ints + [vals[1]]) if kid == spmd.REDUCE_I32 else \
                   (vals + ints + [vals[1]]) if kid == spmd.SCAN_I32 else (vals + ints)
            items.append(B.BatchItem(kid, n, 1, bd, vals[0].value, vals[1].value))
        ptrs = (C.c_void_p * len(args))(*[C.cast(C.pointer(a), C.c_void_p).value for a in args])
        keep.append((args, ptrs))
        descs.append(B.LaunchDesc(kid, (C.c_uint32 * 3)(4, 1, 1), (C.c_uint32 * 3)(bd, 1, 1), 0,
                                  C.cast(ptrs, C.POINTER(C.c_void_p))))
    lib = spmd.lib()
    darr = (B.LaunchDesc * len(descs))(*descs)
    bound = lib.spmd_launch_batch_workspace_size(darr, len(descs))
    assert bound > 0
    iarr = (B.BatchItem * len(items))(*items)
    for c in cands:
        sch = (B.Schedule * len(items))(*[B.Schedule(*c) for _ in items])
        need = lib.spmd_batch_workspace_size(iarr, sch, len(items))
        if need == 0:  # candidate invalid for a class (JACOBI items > 8; items > 16 scan only)
            assert c[1] > 8
            continue
        assert need <= bound, (c, need, bound)
    # and for a random mix of per-launch schedules
    for _ in range(50):
        pick = [cands[int(j)] for j in rng.integers(0, len(cands), len(items))]
        pick = [(b, min(it, 8) if items[k].kernel_id == spmd.JACOBI5_F32 else
                 it if items[k].kernel_id == spmd.SCAN_I32 else min(it, 16), f)
                for k, (b, it, f) in enumerate(pick)]
        sch = (B.Schedule * len(items))(*[B.Schedule(*c) for c in pick])
        need = lib.spmd_batch_workspace_size(iarr, sch, len(items))
        assert 0 < need <= bound


def test_batch_dependencies_validated_on_host(spmd):
    """dep[i] must name an earlier instance, in any queue; anything else is
    refused before any device work."""
    import ctypes as C

    from paper_2206_07896_amd import batch as B

    p = [0x10000, 0x20000, 0x30000]
    items = (B.BatchItem * 3)(B.BatchItem(spmd.SCAN_I32, 1000, 1, 256, p[0], p[1]),
                              B.BatchItem(spmd.HIST256_U32, 1000, 1, 256, p[1], p[2]),
                              B.BatchItem(spmd.SCAN_I32, 1000, 1, 256, p[1], p[0]))
    sch = (B.Schedule * 3)(*[B.Schedule(256, 4, 1)] * 3)
    lib = spmd.lib()

    def size(deps):
        d = (C.c_uint32 * 3)(*[B.NO_DEP if v is None else v for v in deps])
        return lib.spmd_batch_workspace_size_dep(items, sch, d, 3)

    base = lib.spmd_batch_workspace_size(items, sch, 3)
    assert base > 0
    assert size([None, None, None]) == base           # no dependency: the plain plan
    assert size([None, 0, None]) > 0                   # SCAN -> HIST
    assert size([None, None, 0]) > 0                   # same queue, next level
    assert size([None, None, 1]) > 0                   # HIST -> SCAN
    assert size([None, 0, 1]) > 0                      # three levels
    assert size([0, None, None]) == 0                  # itself
    assert size([None, 2, None]) == 0                  # a later instance


def test_sched_chunks_closed_forms(spmd):
    """Chunk counts per candidate: ceil(blocks / bpf), SCAN one tile per
    chunk, 2^32 - 1 where the candidate is invalid for the class."""
    from paper_2206_07896_amd import learned as L

    specs = [{"kid": spmd.REDUCE_I32, "nx": 100000, "ny": 1, "block_dim": 256},
             {"kid": spmd.SCAN_I32, "nx": 100000, "ny": 1, "block_dim": 256},
             {"kid": spmd.JACOBI5_F32, "nx": 300, "ny": 200, "block_dim": 128}]
    ch = L.sched_chunks(specs)
    C = L.CANDIDATES
    assert ch.shape == (3, len(C))
    for j, (blk, it, bpf) in enumerate(C):
        nb = -(-100000 // (blk * it))
        if it > 16:
            assert ch[0, j] == 0xFFFFFFFF                       # 32 items: scan only
        else:
            assert ch[0, j] == -(-nb // bpf), (blk, it, bpf)
        assert ch[1, j] == nb                                   # scan: one tile per chunk
        if it > 8:
            assert ch[2, j] == 0xFFFFFFFF                       # Jacobi takes at most 8 cells per thread
        else:
            nbj = -(-300 // 64) * -(-200 // ((blk // 64) * it))  # 64-column blocks of blk/64 rows x it cells
            assert ch[2, j] == -(-nbj // bpf)


def test_batch_rejects_output_over_input(spmd):
    """An instance's output may not overlap its input (the plan may run it
    more than once): refused on the host for every batchable class, while
    adjacent buffers are accepted."""
    from paper_2206_07896_amd import batch as B

    lib = spmd.lib()
    base = 0x100000

    def ok(kid, n, ny, inp, out):
        items = (B.BatchItem * 1)(B.BatchItem(kid, n, ny, 256, inp, out))
        sch = (B.Schedule * 1)(B.Schedule(256, 4, 1))
        return lib.spmd_batch_workspace_size(items, sch, 1) > 0

    n = 1000
    for kid, ny, out_bytes in ((spmd.SCAN_I32, 1, 4 * n), (spmd.REDUCE_I32, 1, 4), (spmd.HIST256_U32, 1, 1024),
                               (spmd.JACOBI5_F32, 20, 4 * n * 20)):
        in_bytes = 4 * n * ny
        assert not ok(kid, n, ny, base, base), kid                            # in place
        assert not ok(kid, n, ny, base, base + in_bytes - 4), kid             # output starts inside the input
        assert not ok(kid, n, ny, base + out_bytes - 4, base), kid            # input starts inside the output
        assert ok(kid, n, ny, base, base + in_bytes), kid                     # adjacent after
        assert ok(kid, n, ny, base + out_bytes, base), kid                    # adjacent before
