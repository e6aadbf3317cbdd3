"""spmd_launch_batch (CUDA-style launch descriptors run as one batch of the
block queue) on the GPU: as-launched schedules, the learned schedule and its
exhaustive fallback, against the oracle."""

import numpy as np
import pytest

from test_gpu_batch import check_all, make_instances, say, scribble

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def spmd():
    import torch

    assert torch.cuda.is_available()
    import paper_2206_07896_amd as m

    yield m
    m.batch._lib.spmd_model_load(None, 0, None, 0.0)  # unload


def descs_of(spmd, insts):
    """Each instance as the launch a CUDA program would make: its blockDim
    and a grid covering its elements with the instance's items per thread."""
    import torch

    out = []
    for it in insts:
        bd, items, _ = it["sched"]
        if it["kind"] == "jacobi":
            by = bd // 64
            grid = (-(-it["n"] // 64), max(1, -(-it["ny"] // (by * items))))
            out.append((spmd.JACOBI5_F32, grid, (64, by), 0, [it["tin"], it["tout"], it["n"], it["ny"]]))
            continue
        grid = (max(1, -(-it["n"] // (bd * items))),)
        if it["kind"] == "reduce":
            part = torch.empty(1, dtype=torch.int32, device="cuda")
            it["_keep"] = part
            out.append((spmd.REDUCE_I32, grid, (bd,), 4 * bd, [it["tin"], part, it["tout"], it["n"], part]))
        elif it["kind"] == "scan":
            out.append((spmd.SCAN_I32, grid, (bd,), 0, [it["tin"], it["tout"], it["n"], it["tin"]]))
        else:
            out.append((spmd.HIST256_U32, grid, (bd,), 0, [it["tin"], it["tout"], it["n"]]))
    return out


def test_as_launched_matches_oracle(spmd):
    say("launch_batch as launched, 120 instances")
    insts = make_instances(spmd, 120, 11)
    descs = descs_of(spmd, insts)
    scribble(insts)
    ws = spmd.batch.launch_batch(descs, spmd.batch.SCHED_AS_LAUNCHED)
    spmd.sync()
    check_all(insts, "as launched")
    # the same workspace again: the call waits for the stream before reusing it
    scribble(insts)
    spmd.batch.launch_batch(descs, spmd.batch.SCHED_AS_LAUNCHED, workspace=ws)
    spmd.batch.launch_batch(descs, spmd.batch.SCHED_AS_LAUNCHED, workspace=ws)
    spmd.sync()
    check_all(insts, "as launched, reused workspace")
    rep = spmd.batch.launch_batch_report()
    assert rep["launches"] == len(insts) and rep["by_model"] == 0


def test_learned_without_model_is_an_error(spmd):
    spmd.batch._lib.spmd_model_load(None, 0, None, 0.0)
    insts = make_instances(spmd, 4, 12)
    with pytest.raises(spmd.SpmdError):
        spmd.batch.launch_batch(descs_of(spmd, insts), spmd.batch.SCHED_LEARNED)


def test_learned_and_fallback_match_oracle(spmd):
    from oracle import mlp as omlp

    insts = make_instances(spmd, 24, 13, nmax_log2=12)
    descs = descs_of(spmd, insts)
    params = np.stack([omlp.init_params(s) for s in (1, 2, 3)]).astype(np.float32)
    norm = np.concatenate([np.zeros(12), np.ones(12)]).astype(np.float32)
    say("launch_batch learned, model always confident")
    spmd.batch.model_load(params, norm, float("inf"))
    scribble(insts)
    spmd.batch.launch_batch(descs, spmd.batch.SCHED_LEARNED)
    spmd.sync()
    check_all(insts, "learned")
    rep = spmd.batch.launch_batch_report()
    assert rep == {"launches": 24, "by_model": 24, "tuned": 0, "cached": 0}
    say("launch_batch learned, model never confident: exhaustive fallback")
    spmd.batch.model_load(params, norm, -1.0)
    scribble(insts)
    spmd.batch.launch_batch(descs, spmd.batch.SCHED_LEARNED)
    spmd.sync()
    check_all(insts, "fallback tuned")
    keys = {(it["kid"], it["n"], it["ny"], it["bd"]) for it in insts}
    rep = spmd.batch.launch_batch_report()
    assert rep["by_model"] == 0 and rep["tuned"] == len(keys) and rep["tuned"] + rep["cached"] == 24
    scribble(insts)
    spmd.batch.launch_batch(descs, spmd.batch.SCHED_LEARNED)
    spmd.sync()
    check_all(insts, "fallback cached")
    rep = spmd.batch.launch_batch_report()
    assert rep["cached"] == 24 and rep["tuned"] == 0
    spmd.batch._lib.spmd_model_load(None, 0, None, 0.0)


def test_model_batch_slack(spmd):
    """spmd_model_batch_slack sets the loaded model's batch-aware slack:
    refused without a model or for a negative or non-finite slack; with a
    model, learned batches at slacks from 0 (least predicted time only) to
    2 (up to 3x the least) all match the oracle."""
    from oracle import mlp as omlp

    lib = spmd.batch._lib
    lib.spmd_model_load(None, 0, None, 0.0)
    assert lib.spmd_model_batch_slack(0.5) == -4  # no model loaded
    params = np.stack([omlp.init_params(s) for s in (4, 5)]).astype(np.float32)
    norm = np.concatenate([np.zeros(12), np.ones(12)]).astype(np.float32)
    spmd.batch.model_load(params, norm, float("inf"))
    for bad in (-0.1, float("nan"), float("inf")):
        assert lib.spmd_model_batch_slack(bad) == -4
    insts = make_instances(spmd, 16, 14, nmax_log2=12)
    descs = descs_of(spmd, insts)
    for slack in (0.0, 0.2, 2.0):
        say("launch_batch learned, slack", slack)
        spmd.batch.model_load(params, norm, float("inf"), slack)
        scribble(insts)
        spmd.batch.launch_batch(descs, spmd.batch.SCHED_LEARNED)
        spmd.sync()
        check_all(insts, f"slack {slack}")
    lib.spmd_model_load(None, 0, None, 0.0)
