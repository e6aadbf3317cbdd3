"""Schedule choice for batched launches: exhaustive autotuning and the
learned cost model.

A schedule is (block, items, bpf): threads per logical block, elements per
thread (cells per thread for the stencil) and logical blocks per queue
fetch.  The paper sets the blocks per fetch by heuristics -- average
fetching, ceil(grid / pool), or a larger grain found by hand (Section IV-A)
-- and notes that the best grain depends on the kernel.  Here:

* the autotuner measures an instance under every candidate schedule
  (spmd_tune.h) -- exhaustive, exact, slow;
* the cost model (spmd_mlp.h) is an ensemble of small MLPs trained on the
  autotuner's timings by the library's own forward/backward/Adam kernels;
  it predicts log time for every candidate of a launch in one inference
  kernel, picks the argmin, and flags launches where the ensemble
  disagrees (standard deviation above a threshold) for the exhaustive
  fallback.

Launch features (the 9 model inputs besides the schedule) describe the
instance as its CUDA source would be written for its blockDim: the class
one-hot, log2 n, log2 blockDim, log2 of the block's shared-memory bytes,
the barriers per block and the warp-level operations per warp.
"""

from __future__ import annotations

import ctypes
import json
import math
import os

import numpy as np
import torch

from . import HIST256_U32, JACOBI5_F32, REDUCE_I32, SCAN_I32, _check, _lib, _stream_handle
from . import batch as B

NFEAT, NSCHED, DIN, NPARAM = 9, 3, 12, 12 * 64 + 64 + 64 * 64 + 64 + 64 + 1
KIND_IDS = (REDUCE_I32, SCAN_I32, HIST256_U32, JACOBI5_F32)
# the library's candidate table: block 64..512, items 1..32 (32: scan tiles only), bpf 1..32
CANDIDATES = B.sched_candidates()
BLOCKS = tuple(sorted({b for b, _, _ in CANDIDATES}))

_P = ctypes.c_void_p
_lib.spmd_mlp_forward.argtypes = [_P, _P, _P, ctypes.c_uint32, _P, _P, _P, _P]
_lib.spmd_mlp_workspace_size.argtypes = [ctypes.c_uint32]
_lib.spmd_mlp_workspace_size.restype = ctypes.c_size_t
_lib.spmd_mlp_backward.argtypes = [_P, _P, _P, _P, ctypes.c_uint32, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]
_lib.spmd_mlp_adam.argtypes = [_P, _P, _P, _P, ctypes.c_uint32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                               ctypes.c_float, _P]
_lib.spmd_mlp_choose.argtypes = [_P, ctypes.c_uint32, _P, _P, ctypes.c_uint32, _P, ctypes.c_uint32, _P, _P, _P, _P, _P]
_lib.spmd_mlp_choose_batch.argtypes = [_P, ctypes.c_uint32, _P, _P, ctypes.c_uint32, _P, ctypes.c_uint32, _P, _P,
                                       ctypes.c_float, _P, _P, _P, _P]
_lib.spmd_mlp_choose_batch.restype = ctypes.c_int
_lib.spmd_sched_chunks.argtypes = [ctypes.POINTER(B.BatchItem), ctypes.c_int, _P]
_lib.spmd_sched_chunks.restype = ctypes.c_int
BATCH_SLACK = 0.2  # SPMD_BATCH_SLACK, the library's default
SLACK_CHOICES = (0.1, 0.2, 0.3, 0.5, 1.0, 2.0)  # tried on held-out launches for each trained model
for _f in ("spmd_mlp_forward", "spmd_mlp_backward", "spmd_mlp_adam", "spmd_mlp_choose"):
    getattr(_lib, _f).restype = ctypes.c_int
_lib.spmd_tune_workspace_size.argtypes = [ctypes.POINTER(B.BatchItem), ctypes.POINTER(B.Schedule), ctypes.c_int]
_lib.spmd_tune_workspace_size.restype = ctypes.c_size_t
_lib.spmd_tune_time.argtypes = [ctypes.POINTER(B.BatchItem), ctypes.POINTER(B.Schedule), ctypes.c_int,
                                ctypes.c_uint32, _P, ctypes.c_size_t, _P, ctypes.POINTER(ctypes.c_float)]
_lib.spmd_tune_time.restype = ctypes.c_int


# ---------------------------------------------------------------------------
# features
# ---------------------------------------------------------------------------

def candidate_inputs() -> np.ndarray:
    return np.array([[math.log2(b), math.log2(it), math.log2(f)] for b, it, f in CANDIDATES], np.float32)


def valid_candidates(kid: int) -> np.ndarray:
    """Jacobi takes at most 8 cells per thread; 32 items are scan tiles
    only."""
    return np.array([not ((kid == JACOBI5_F32 and it > 8) or (kid != SCAN_I32 and it > 16))
                     for _, it, _ in CANDIDATES], bool)


def launch_features(spec) -> np.ndarray:
    """The 9 launch features of a mixed-workload spec, as the library
    computes them (spmd_sched_features)."""
    return np.array(B.sched_features(spec["kid"], spec["nx"], spec["ny"], spec["block_dim"]), np.float32)


def heuristic_schedule(spec, pools) -> tuple:
    """The method without the learned part: the instance's own blockDim,
    4 items per thread and the paper's average coarse-grained fetching."""
    items = 4
    nb = B.item_blocks(spec["kid"], spec["nx"], spec["ny"], spec["block_dim"], items)
    return (spec["block_dim"], items, B.average_bpf(nb, pools[(spec["kid"], spec["block_dim"])]))


def pools_for(workers_per_cu: int = 0):
    return {(k, b): B.pool_size(k, b, workers_per_cu) for k in KIND_IDS for b in BLOCKS}


# ---------------------------------------------------------------------------
# exhaustive autotuner
# ---------------------------------------------------------------------------

class Autotuner:
    """Times instances under candidate schedules with spmd_tune_time and
    keeps an append-only record (one JSON line per measurement)."""

    def __init__(self, reps: int = 3, db_path: str | None = None):
        self.reps = reps
        self.db_path = db_path
        self._ws = None

    def _workspace(self, nbytes):
        if self._ws is None or self._ws.numel() < nbytes + 256:
            self._ws = torch.empty(max(nbytes, 1 << 20) * 2 + 256, dtype=torch.uint8, device="cuda")
        off = (-self._ws.data_ptr()) % 256
        return self._ws.data_ptr() + off, self._ws.numel() - off

    def time(self, item_tuple, schedules):
        """Milliseconds of one instance (kid, n, ny, block_dim, in, out) under
        each schedule (fastest of `reps` runs after a warm-up)."""
        kid, n, ny, bd, tin, tout = item_tuple
        it = B.BatchItem(int(kid), int(n), int(ny), int(bd), tin.data_ptr(), tout.data_ptr())
        ns = len(schedules)
        arr = (B.Schedule * ns)(*[B.Schedule(*map(int, s)) for s in schedules])
        need = int(_lib.spmd_tune_workspace_size(ctypes.byref(it), arr, ns))
        if need == 0:
            raise ValueError("invalid schedule for this instance")
        ptr, size = self._workspace(need)
        out = (ctypes.c_float * ns)()
        _check(_lib.spmd_tune_time(ctypes.byref(it), arr, ns, self.reps, ptr, size, _stream_handle(None), out),
               "spmd_tune_time")
        return np.array(out[:], np.float64)

    def sweep(self, specs, data, progress=None):
        """Exhaustive timings: [len(specs), len(CANDIDATES)] ms, NaN where
        a candidate is invalid for the class.  `progress` (a print-like
        function) is called every 200 launches."""
        items = data.items()
        T = np.full((len(specs), len(CANDIDATES)), np.nan)
        f = open(self.db_path, "a") if self.db_path else None
        for i, s in enumerate(specs):
            ok = valid_candidates(s["kid"])
            idx = np.nonzero(ok)[0]
            ms = self.time(items[i], [CANDIDATES[j] for j in idx])
            T[i, idx] = ms
            if f is not None:
                f.write(json.dumps({"kid": s["kid"], "n": s["n"], "nx": s["nx"], "ny": s["ny"],
                                    "block_dim": s["block_dim"],
                                    "ms": [None if np.isnan(v) else float(v) for v in T[i]]}) + "\n")
            if progress is not None and i % 200 == 0:
                progress(f"  tuned {i}/{len(specs)}")
        if f is not None:
            f.close()
        return T


# ---------------------------------------------------------------------------
# the learned cost model
# ---------------------------------------------------------------------------

def _f32(t):
    return t.contiguous().to(torch.float32)


class CostModel:
    """An ensemble of K MLPs (spmd_mlp.h) with one input normalisation."""

    def __init__(self, params: np.ndarray, norm: np.ndarray):
        self.params = np.asarray(params, np.float32).reshape(-1, NPARAM)
        self.norm = np.asarray(norm, np.float32).reshape(2 * DIN)
        self.k = self.params.shape[0]
        self.tau = float("inf")  # ensemble spread above which the exhaustive fallback runs
        self.slack = BATCH_SLACK  # of the batch-aware choice (SPMD_SCHED_LEARNED)
        self._dev = None

    def device_tensors(self):
        if self._dev is None:
            self._dev = (torch.from_numpy(self.params.reshape(-1).copy()).cuda(),
                         torch.from_numpy(self.norm.copy()).cuda())
        return self._dev

    def to_json(self) -> str:
        return json.dumps({"k": self.k, "tau": self.tau, "slack": self.slack, "norm": self.norm.tolist(),
                           "params": self.params.tolist()})

    @staticmethod
    def from_json(text: str) -> "CostModel":
        d = json.loads(text)
        m = CostModel(np.array(d["params"], np.float32), np.array(d["norm"], np.float32))
        m.tau = float(d.get("tau", float("inf")))
        m.slack = float(d.get("slack", BATCH_SLACK))
        return m

    def load(self) -> None:
        """Load this model into the library for SPMD_SCHED_LEARNED on the
        current device (its fallback threshold and batch slack with it)."""
        B.model_load(self.params, self.norm, self.tau, self.slack)

    def predict(self, X: np.ndarray, model: int = 0) -> np.ndarray:
        """Predicted log-microseconds of rows X[n x 12] under one model."""
        p, nm = self.device_tensors()
        x = torch.from_numpy(np.ascontiguousarray(X, np.float32)).cuda()
        y = torch.empty(x.shape[0], dtype=torch.float32, device="cuda")
        _check(_lib.spmd_mlp_forward(p.data_ptr() + 4 * NPARAM * model, nm.data_ptr(), x.data_ptr(), x.shape[0],
                                     y.data_ptr(), None, None, _stream_handle(None)), "spmd_mlp_forward")
        return y.cpu().numpy()

    def choose(self, specs, slack=None):
        """(candidate index, predicted log-us, ensemble sd) per spec, by the
        inference kernel: the least predicted time per launch, or with
        `slack` the batch-aware choice (spmd_mlp_choose_batch: fewest chunks
        within ln(1 + slack) of the least)."""
        p, nm = self.device_tensors()
        m = len(specs)
        feats = torch.from_numpy(np.stack([launch_features(s) for s in specs])).cuda()
        cands = torch.from_numpy(candidate_inputs()).cuda()
        valid = torch.from_numpy(np.stack([valid_candidates(s["kid"]) for s in specs]).astype(np.uint8)).cuda()
        best = torch.empty(m, dtype=torch.int32, device="cuda")
        pred = torch.empty(m, dtype=torch.float32, device="cuda")
        sd = torch.empty(m, dtype=torch.float32, device="cuda")
        if slack is None:
            _check(_lib.spmd_mlp_choose(p.data_ptr(), self.k, nm.data_ptr(), feats.data_ptr(), m, cands.data_ptr(),
                                        len(CANDIDATES), valid.data_ptr(), best.data_ptr(), pred.data_ptr(),
                                        sd.data_ptr(), _stream_handle(None)), "spmd_mlp_choose")
        else:
            ch = torch.from_numpy(sched_chunks(specs).view(np.int32)).cuda()
            _check(_lib.spmd_mlp_choose_batch(p.data_ptr(), self.k, nm.data_ptr(), feats.data_ptr(), m,
                                              cands.data_ptr(), len(CANDIDATES), valid.data_ptr(), ch.data_ptr(),
                                              float(slack), best.data_ptr(), pred.data_ptr(), sd.data_ptr(),
                                              _stream_handle(None)), "spmd_mlp_choose_batch")
        return best.cpu().numpy().astype(np.int64), pred.cpu().numpy(), sd.cpu().numpy()


def sched_chunks(specs) -> np.ndarray:
    """Chunk counts [len(specs) x candidates] (spmd_sched_chunks); 2^32 - 1
    where a candidate is invalid for the launch."""
    m = len(specs)
    arr = (B.BatchItem * max(m, 1))()
    for i, s in enumerate(specs):
        arr[i] = B.BatchItem(int(s["kid"]), int(s["nx"]), int(s["ny"]), int(s["block_dim"]), None, None)
    out = np.zeros((m, len(CANDIDATES)), np.uint32)
    _check(_lib.spmd_sched_chunks(arr, m, out.ctypes.data), "spmd_sched_chunks")
    return out


def training_rows(specs, T):
    """Model rows (features + schedule inputs) and targets log(us) for every
    measured (spec, candidate)."""
    ci = candidate_inputs()
    X, t = [], []
    for i, s in enumerate(specs):
        f = launch_features(s)
        for j in np.nonzero(np.isfinite(T[i]))[0]:
            X.append(np.concatenate([f, ci[j]]))
            t.append(math.log(max(T[i, j], 1e-6) * 1e3))
    return np.array(X, np.float32), np.array(t, np.float32)


def init_params(seed: int) -> np.ndarray:
    """He-style initial weights from a seeded generator, biases zero (the
    layout of spmd_mlp.h)."""
    rng = np.random.default_rng(seed)
    parts = [rng.standard_normal(DIN * 64) * math.sqrt(2.0 / DIN), np.zeros(64),
             rng.standard_normal(64 * 64) * math.sqrt(2.0 / 64), np.zeros(64),
             rng.standard_normal(64) * math.sqrt(1.0 / 64), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)


def train(X: np.ndarray, t: np.ndarray, k_models: int = 3, steps: int = 3000, lr: float = 3e-3, seed: int = 0xC5,
          log_every: int = 0):
    """Full-batch Adam on the GPU kernels; returns (CostModel, final losses)."""
    mu = X.mean(axis=0)
    sd = X.std(axis=0)
    inv_sd = np.where(sd > 1e-6, 1.0 / np.maximum(sd, 1e-6), 1.0)
    norm = np.concatenate([mu, inv_sd]).astype(np.float32)
    n = X.shape[0]
    x = torch.from_numpy(np.ascontiguousarray(X, np.float32)).cuda()
    tt = torch.from_numpy(np.ascontiguousarray(t, np.float32)).cuda()
    nm = torch.from_numpy(norm).cuda()
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    h1 = torch.empty(64 * n, dtype=torch.float32, device="cuda")
    h2 = torch.empty(64 * n, dtype=torch.float32, device="cuda")
    ws = torch.empty(int(_lib.spmd_mlp_workspace_size(n)), dtype=torch.uint8, device="cuda")
    grad = torch.empty(NPARAM, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    s = _stream_handle(None)
    out, losses, first = [], [], []
    for k in range(k_models):
        p = torch.from_numpy(init_params(seed + 7919 * k)).cuda()
        m = torch.zeros(NPARAM, dtype=torch.float32, device="cuda")
        v = torch.zeros(NPARAM, dtype=torch.float32, device="cuda")
        for step in range(1, steps + 1):
            _check(_lib.spmd_mlp_forward(p.data_ptr(), nm.data_ptr(), x.data_ptr(), n, y.data_ptr(), h1.data_ptr(),
                                         h2.data_ptr(), s), "spmd_mlp_forward")
            _check(_lib.spmd_mlp_backward(p.data_ptr(), nm.data_ptr(), x.data_ptr(), tt.data_ptr(), n, y.data_ptr(),
                                          h1.data_ptr(), h2.data_ptr(), grad.data_ptr(), loss.data_ptr(),
                                          ws.data_ptr(), ws.numel(), s), "spmd_mlp_backward")
            _check(_lib.spmd_mlp_adam(p.data_ptr(), grad.data_ptr(), m.data_ptr(), v.data_ptr(), step, lr, 0.9, 0.999,
                                      1e-8, s), "spmd_mlp_adam")
            if step == 1:
                first.append(float(loss.item()))
            if log_every and step % log_every == 0:
                print(f"  model {k} step {step} loss {float(loss.item()):.4f}", flush=True)
        # the loss of the final parameters
        _check(_lib.spmd_mlp_forward(p.data_ptr(), nm.data_ptr(), x.data_ptr(), n, y.data_ptr(), h1.data_ptr(),
                                     h2.data_ptr(), s), "spmd_mlp_forward")
        _check(_lib.spmd_mlp_backward(p.data_ptr(), nm.data_ptr(), x.data_ptr(), tt.data_ptr(), n, y.data_ptr(),
                                      h1.data_ptr(), h2.data_ptr(), grad.data_ptr(), loss.data_ptr(),
                                      ws.data_ptr(), ws.numel(), s), "spmd_mlp_backward")
        losses.append(float(loss.item()))
        out.append(p.cpu().numpy())
    model = CostModel(np.stack(out), norm)
    model.initial_losses = first
    return model, losses


def select_batch_slack(model, specs, items, slacks=SLACK_CHOICES, reps=10, log=None):
    """The batch-aware slack for `model`: each slack's choice for the
    launches `specs` (with their device items) is run as one batch replayed
    from a hipGraph (median of `reps` replays); the fastest slack wins.
    Returns (slack, {slack: ms})."""
    table = {}
    for slack in slacks:
        choice = model.choose(specs, slack=slack)[0]
        b = B.Batch(items, [CANDIDATES[j] for j in choice])
        try:
            table[slack] = round(_median_graph_ms(b, reps), 4)
        finally:
            b.close()
        if log is not None:
            log(f"  slack {slack}: {table[slack]:.3f} ms")
    best = min(table, key=lambda k: (table[k], k))
    return best, table


def regret(T, choice):
    """Per-launch (t_chosen - t_best) / t_best from exhaustive timings."""
    best = np.nanmin(T, axis=1)
    chosen = T[np.arange(T.shape[0]), choice]
    return (chosen - best) / best


# ---------------------------------------------------------------------------
# evaluation: exhaustive ground truth, training, held-out regret
# ---------------------------------------------------------------------------

def _median_graph_ms(batch, reps):
    batch.graph_launch()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        batch.graph_launch()
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def evaluate(train_count=500, heldout_count=2000, k_models=3, steps=2000, lr=3e-3, reps=2, fallback_quantile=0.9,
             batch_reps=10, log=print, log2_hi=22.0):
    """Exhaustively time `train_count` launches drawn like the mixed
    workload (seed SEED_TRAIN) under every candidate schedule, train the
    ensemble on the GPU, then choose schedules for `heldout_count` fresh
    launches (seed SEED_HELDOUT) and score the choice against their own
    exhaustive timings.  The fallback threshold is the `fallback_quantile`
    of the ensemble spread over the training launches' choices; held-out
    launches above it take the exhaustive choice."""
    import time

    import synth

    from . import workload as W

    pools = pools_for()
    tuner = Autotuner(reps=reps)
    t0 = time.perf_counter()
    specs_tr = W.mixed_specs(train_count, seed=synth.SEED_TRAIN, log2_hi=log2_hi)
    data_tr = W.MixedData(specs_tr)
    log(f"c5: tuning {train_count} training launches x {len(CANDIDATES)} schedules")
    T_tr = tuner.sweep(specs_tr, data_tr, progress=log)
    del data_tr
    t_tune_tr = time.perf_counter() - t0
    X, t = training_rows(specs_tr, T_tr)
    t1 = time.perf_counter()
    model, losses = train(X, t, k_models=k_models, steps=steps, lr=lr)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    log(f"c5: trained {k_models} models on {X.shape[0]} rows in {t_train:.1f} s, final losses {losses}")
    _, _, sd_tr = model.choose(specs_tr)
    tau = float(np.quantile(sd_tr, fallback_quantile))

    specs_ho = W.mixed_specs(heldout_count, seed=synth.SEED_HELDOUT, log2_hi=log2_hi)
    data_ho = W.MixedData(specs_ho)
    log(f"c5: tuning {heldout_count} held-out launches")
    t2 = time.perf_counter()
    T_ho = tuner.sweep(specs_ho, data_ho, progress=log)
    t_tune_ho = time.perf_counter() - t2
    items = data_ho.items()
    heur = [heuristic_schedule(s, pools) for s in specs_ho]
    t_heur = np.array([tuner.time(items[i], [heur[i]])[0] for i in range(heldout_count)])
    t3 = time.perf_counter()
    choice, pred, sd = model.choose(specs_ho)
    torch.cuda.synchronize()
    t_choose = time.perf_counter() - t3
    exhaustive = np.nanargmin(T_ho, axis=1)
    fb = sd > tau
    choice_fb = np.where(fb, exhaustive, choice)
    best = np.nanmin(T_ho, axis=1)
    r_model = regret(T_ho, choice)
    r_fb = regret(T_ho, choice_fb)
    r_heur = (t_heur - best) / best
    # log-time prediction error of the chosen schedules
    chosen_t = T_ho[np.arange(heldout_count), choice]
    pred_err = np.abs(pred - np.log(chosen_t * 1e3))

    def batch_ms(scheds):
        b = B.Batch(items, scheds)
        try:
            return _median_graph_ms(b, batch_reps)
        finally:
            b.close()

    sched_learned = [CANDIDATES[j] for j in choice_fb]
    sched_exh = [CANDIDATES[j] for j in exhaustive]
    choice_ba = model.choose(specs_ho, slack=BATCH_SLACK)[0]  # SPMD_SCHED_LEARNED's rule, no fallback
    chunks_ho = sched_chunks(specs_ho).astype(np.int64)
    ms_learned = batch_ms(sched_learned)
    ms_learned_ba = batch_ms([CANDIDATES[j] for j in choice_ba])
    model.slack, slack_ms = select_batch_slack(model, specs_ho, items, reps=batch_reps, log=log)
    ms_heur = batch_ms(heur)
    ms_exh = batch_ms(sched_exh)
    del data_ho
    torch.cuda.empty_cache()
    per_class = {}
    for k in KIND_IDS:
        sel = np.array([s["kid"] == k for s in specs_ho])
        per_class[W.KIND_NAMES[k]] = {"launches": int(sel.sum()),
                                      "regret_mean": round(float(r_model[sel].mean()), 4),
                                      "regret_heuristic_mean": round(float(r_heur[sel].mean()), 4)}
    res = {
        "train_launches": train_count, "train_rows": int(X.shape[0]), "heldout_launches": heldout_count,
        "candidates": len(CANDIDATES), "models": k_models, "adam_steps": steps,
        "initial_train_mse": [round(v, 5) for v in model.initial_losses],
        "final_train_mse": [round(v, 5) for v in losses],
        "regret_mean": round(float(r_model.mean()), 4),
        "regret_median": round(float(np.median(r_model)), 4),
        "regret_mean_with_fallback": round(float(r_fb.mean()), 4),
        "fallback_rate": round(float(fb.mean()), 4), "fallback_sd_threshold": round(tau, 4),
        "regret_mean_heuristic": round(float(r_heur.mean()), 4),
        "time_sum_ratio_heuristic_over_learned": round(float(t_heur.sum() / T_ho[np.arange(heldout_count), choice_fb].sum()), 3),
        "abs_log_error_chosen_median": round(float(np.median(pred_err)), 4),
        "per_class": per_class,
        "batch_ms_learned": round(ms_learned, 3), "batch_ms_heuristic": round(ms_heur, 3),
        "batch_ms_exhaustive": round(ms_exh, 3), "batch_ms_learned_batch_aware": round(ms_learned_ba, 3),
        "batch_slack": model.slack, "batch_ms_by_slack": {str(k): v for k, v in slack_ms.items()},
        "chunks_learned": int(chunks_ho[np.arange(heldout_count), choice_fb].sum()),
        "chunks_learned_batch_aware": int(chunks_ho[np.arange(heldout_count), choice_ba].sum()),
        "launches_per_s_learned": round(heldout_count / (ms_learned * 1e-3), 1),
        "launches_per_s_heuristic": round(heldout_count / (ms_heur * 1e-3), 1),
        "launches_per_s_exhaustive": round(heldout_count / (ms_exh * 1e-3), 1),
        "seconds": {"tune_train": round(t_tune_tr, 1), "train": round(t_train, 2),
                    "tune_heldout": round(t_tune_ho, 1), "choose_2000": round(t_choose, 4)},
        "heuristic": "instance blockDim, 4 items per thread, average coarse-grained fetching ceil(blocks/pool)",
    }
    log(f"c5: regret {res['regret_mean']:.3f} (with fallback {res['regret_mean_with_fallback']:.3f}, "
        f"rate {res['fallback_rate']:.2f}), heuristic {res['regret_mean_heuristic']:.3f}; batch ms learned "
        f"{ms_learned:.2f} batch-aware {ms_learned_ba:.2f} heuristic {ms_heur:.2f} exhaustive {ms_exh:.2f}")
    model.tau = tau
    return res, model


def heldout_regret(model, count=200, seed=None, reps=2, log2_hi=22.0, log=None):
    """Schedule regret of `model` on `count` launches drawn like the mixed
    workload from `seed` (default: the held-out seed, never trained on),
    each timed in this run under every valid candidate (the exhaustive
    ground truth).  The model picks the least predicted time per launch;
    with the fallback, launches whose ensemble spread exceeds the model's
    threshold take the exhaustive choice instead.  The paper's heuristic
    (blockDim as launched, 4 items per thread, average coarse-grained
    fetching) is timed on the same launches for comparison."""
    import time

    import synth

    from . import workload as W

    seed = synth.SEED_HELDOUT if seed is None else seed
    specs = W.mixed_specs(count, seed=seed, log2_hi=log2_hi)
    data = W.MixedData(specs)
    tuner = Autotuner(reps=reps)
    t0 = time.perf_counter()
    T = tuner.sweep(specs, data, progress=log)
    items = data.items()
    pools = pools_for()
    heur = [heuristic_schedule(s, pools) for s in specs]
    t_heur = np.array([tuner.time(items[i], [heur[i]])[0] for i in range(count)])
    t_tune = time.perf_counter() - t0
    choice, _, sd = model.choose(specs)
    exhaustive = np.nanargmin(T, axis=1)
    fb = sd > model.tau
    best = np.nanmin(T, axis=1)
    r = regret(T, choice)
    r_fb = regret(T, np.where(fb, exhaustive, choice))
    r_heur = (t_heur - best) / best
    del data
    return {
        "heldout_launches": count, "seed": seed, "candidates": len(CANDIDATES),
        "regret_mean": round(float(r.mean()), 4), "regret_median": round(float(np.median(r)), 4),
        "regret_p90": round(float(np.quantile(r, 0.9)), 4),
        "regret_mean_with_fallback": round(float(r_fb.mean()), 4),
        "fallback_rate": round(float(fb.mean()), 4), "fallback_sd_threshold": round(float(model.tau), 4),
        "regret_mean_heuristic": round(float(r_heur.mean()), 4),
        "seconds_exhaustive_timing": round(t_tune, 1),
        "timing": f"fastest of {reps} runs after a warm-up per (launch, schedule), each launch alone in a batch",
    }


MODEL_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cost_model.json")


def load_default():
    """The cost model shipped with the package (trained on MI355X by
    `python -m paper_2206_07896_amd.train`), or None."""
    if not os.path.exists(MODEL_PATH):
        return None
    with open(MODEL_PATH) as f:
        return CostModel.from_json(f.read())


def contention_study(model=None, log2_sizes=(12, 14, 16, 18, 20, 22), reps=5, log=None):
    """Does LDS-atomic contention move a histogram's best schedule?  For
    each size, keys of bounded Zipf exponent 0 (uniform), 1.1 (the workload's),
    2 and 3, and every key in one bin, are timed under every candidate
    schedule.  Per row: the best time and schedule, the regret of the
    schedule that is best at exponent 1.1 (what a model trained on the
    workload would learn), and, with a model, the regret of its choice.
    The launch features carry no key distribution, so these regrets bound
    what a contention feature could recover (Section V-C: the grain size
    depends on the kernel's atomics)."""
    import synth

    tuner = Autotuner(reps=reps)
    valid = np.nonzero(valid_candidates(HIST256_U32))[0]  # indices into CANDIDATES
    cands = [CANDIDATES[j] for j in valid]
    dists = (("zipf0", 0.0), ("zipf1.1", 1.1), ("zipf2", 2.0), ("zipf3", 3.0), ("one bin", None))
    hist = torch.zeros(256, dtype=torch.int32, device="cuda")
    rows = []
    for lg in log2_sizes:
        n = 1 << lg
        keys = torch.empty(n, dtype=torch.int32, device="cuda")
        T = {}
        for name, alpha in dists:
            if alpha is None:
                keys.fill_(7)
            else:
                B.synth_zipf_u32(keys, synth.SEED_HIST ^ lg, torch.from_numpy(synth.zipf_cdf(alpha, 256)).cuda())
            item = (HIST256_U32, n, 1, 256, keys, hist)
            # two full sweeps, the faster of each: at ~10 us a single stall skews one timing
            T[name] = np.minimum(tuner.time(item, cands), tuner.time(item, cands))
        spec = {"kid": HIST256_U32, "n": n, "nx": n, "ny": 1, "block_dim": 256}
        chosen = int(np.nonzero(valid == int(model.choose([spec])[0][0]))[0][0]) if model is not None else None
        ref = int(np.argmin(T["zipf1.1"]))
        for name, _ in dists:
            t = T[name]
            j = int(np.argmin(t))
            row = {"log2_n": lg, "keys": name, "best_us": round(float(t[j]) * 1e3, 2), "best": list(cands[j]),
                   "regret_of_zipf1.1_best": round(float(t[ref] / t[j] - 1.0), 4)}
            if chosen is not None:
                row["model"] = list(cands[chosen])
                row["regret_of_model"] = round(float(t[chosen] / t[j] - 1.0), 4)
            rows.append(row)
            if log is not None:
                log(json.dumps(row))
        del keys
    return rows


def main(argv=None):
    import argparse
    import sys

    ap = argparse.ArgumentParser(description="train and evaluate the schedule cost model on this GPU")
    ap.add_argument("--train-count", type=int, default=500)
    ap.add_argument("--heldout", type=int, default=2000)
    ap.add_argument("--models", type=int, default=3)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--out", default=MODEL_PATH)
    ap.add_argument("--report", default=None)
    ap.add_argument("--select-slack", action="store_true",
                    help="only choose the shipped model's batch-aware slack on the held-out launches and write it back")
    ap.add_argument("--contention", action="store_true",
                    help="only time histograms of skewed keys under every schedule (no training)")
    a = ap.parse_args(argv)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    if a.select_slack:
        import synth

        from . import workload as W

        model = load_default()
        specs = W.mixed_specs(a.heldout, seed=synth.SEED_HELDOUT)
        data = W.MixedData(specs)
        model.slack, table = select_batch_slack(model, specs, data.items(), log=log)
        with open(a.out, "w") as f:
            f.write(model.to_json())
        text = json.dumps({"heldout_launches": a.heldout, "batch_slack": model.slack,
                           "batch_ms_by_slack": {str(k): v for k, v in table.items()}})
        print(text, flush=True)
        if a.report:
            with open(a.report, "w") as f:
                f.write(text + "\n")
        return

    if a.contention:
        rows = contention_study(load_default(), log=log)
        text = json.dumps(rows)
        print(text, flush=True)
        if a.report:
            with open(a.report, "w") as f:
                f.write(text + "\n")
        return

    res, model = evaluate(a.train_count, a.heldout, a.models, a.steps, log=log)
    with open(a.out, "w") as f:
        f.write(model.to_json())
    text = json.dumps(res)
    print(text, flush=True)
    if a.report:
        with open(a.report, "w") as f:
            f.write(text + "\n")


if __name__ == "__main__":
    main()
