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

import numpy as np
import torch

from . import HIST256_U32, JACOBI5_F32, REDUCE_I32, SCAN_I32, _check, _lib, _stream_handle
from . import batch as B

NFEAT, NSCHED, DIN, NPARAM = 9, 3, 12, 12 * 64 + 64 + 64 * 64 + 64 + 64 + 1
KIND_IDS = (REDUCE_I32, SCAN_I32, HIST256_U32, JACOBI5_F32)
BLOCKS = (64, 128, 256, 512)
ITEMS = (1, 2, 4, 8, 16)
BPFS = (1, 2, 4, 8, 16, 32)
CANDIDATES = [(b, it, f) for b in BLOCKS for it in ITEMS for f in BPFS]

_P = ctypes.c_void_p
_lib.spmd_mlp_forward.argtypes = [_P, _P, _P, ctypes.c_uint32, _P, _P, _P, _P]
_lib.spmd_mlp_workspace_size.argtypes = [ctypes.c_uint32]
_lib.spmd_mlp_workspace_size.restype = ctypes.c_size_t
_lib.spmd_mlp_backward.argtypes = [_P, _P, _P, _P, ctypes.c_uint32, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]
_lib.spmd_mlp_adam.argtypes = [_P, _P, _P, _P, ctypes.c_uint32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                               ctypes.c_float, _P]
_lib.spmd_mlp_choose.argtypes = [_P, ctypes.c_uint32, _P, _P, ctypes.c_uint32, _P, ctypes.c_uint32, _P, _P, _P, _P, _P]
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
    return np.array([not (kid == JACOBI5_F32 and it > 8) for _, it, _ in CANDIDATES], bool)


def launch_features(spec) -> np.ndarray:
    """The 9 launch features of a mixed-workload spec (see module doc)."""
    kid, bd, n = spec["kid"], spec["block_dim"], max(1, spec["n"])
    onehot = [1.0 if kid == k else 0.0 for k in KIND_IDS]
    if kid == REDUCE_I32:
        shm, bar, wops = 4 * bd, math.log2(bd) + 1, 0
    elif kid == SCAN_I32:
        shm, bar, wops = 4 * (bd // 32) + 4, 2, 10
    elif kid == HIST256_U32:
        shm, bar, wops = 1024, 2, 0
    else:
        shm, bar, wops = 4 * (bd // 64 + 2) * 66, 1, 0
    return np.array(onehot + [math.log2(n), math.log2(bd), math.log2(shm), bar, wops], np.float32)


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

    def sweep(self, specs, data, record=None):
        """Exhaustive timings: [len(specs), len(CANDIDATES)] ms, NaN where
        a candidate is invalid for the class."""
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
                                    "block_dim": s["block_dim"], "ms": [float(v) for v in T[i]],
                                    **(record or {})}) + "\n")
            if record is not None and i % 200 == 0:
                print(f"  tuned {i}/{len(specs)}", flush=True)
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
        self._dev = None

    def device_tensors(self):
        if self._dev is None:
            self._dev = (torch.from_numpy(self.params.reshape(-1).copy()).cuda(),
                         torch.from_numpy(self.norm.copy()).cuda())
        return self._dev

    def to_json(self) -> str:
        return json.dumps({"k": self.k, "norm": self.norm.tolist(), "params": self.params.tolist()})

    @staticmethod
    def from_json(text: str) -> "CostModel":
        d = json.loads(text)
        return CostModel(np.array(d["params"], np.float32), np.array(d["norm"], np.float32))

    def predict(self, X: np.ndarray, model: int = 0) -> np.ndarray:
        """Predicted log-microseconds of rows X[n x 12] under one model."""
        p, nm = self.device_tensors()
        x = torch.from_numpy(np.ascontiguousarray(X, np.float32)).cuda()
        y = torch.empty(x.shape[0], dtype=torch.float32, device="cuda")
        _check(_lib.spmd_mlp_forward(p.data_ptr() + 4 * NPARAM * model, nm.data_ptr(), x.data_ptr(), x.shape[0],
                                     y.data_ptr(), None, None, _stream_handle(None)), "spmd_mlp_forward")
        return y.cpu().numpy()

    def choose(self, specs):
        """(candidate index, predicted log-us, ensemble sd) per spec, by the
        inference kernel."""
        p, nm = self.device_tensors()
        m = len(specs)
        feats = torch.from_numpy(np.stack([launch_features(s) for s in specs])).cuda()
        cands = torch.from_numpy(candidate_inputs()).cuda()
        valid = torch.from_numpy(np.stack([valid_candidates(s["kid"]) for s in specs]).astype(np.uint8)).cuda()
        best = torch.empty(m, dtype=torch.int32, device="cuda")
        pred = torch.empty(m, dtype=torch.float32, device="cuda")
        sd = torch.empty(m, dtype=torch.float32, device="cuda")
        _check(_lib.spmd_mlp_choose(p.data_ptr(), self.k, nm.data_ptr(), feats.data_ptr(), m, cands.data_ptr(),
                                    len(CANDIDATES), valid.data_ptr(), best.data_ptr(), pred.data_ptr(),
                                    sd.data_ptr(), _stream_handle(None)), "spmd_mlp_choose")
        return best.cpu().numpy().astype(np.int64), pred.cpu().numpy(), sd.cpu().numpy()


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
    out, losses = [], []
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
            if log_every and step % log_every == 0:
                print(f"  model {k} step {step} loss {float(loss.item()):.4f}", flush=True)
        losses.append(float(loss.item()))
        out.append(p.cpu().numpy())
    return CostModel(np.stack(out), norm), losses


def regret(T, choice):
    """Per-launch (t_chosen - t_best) / t_best from exhaustive timings."""
    best = np.nanmin(T, axis=1)
    chosen = T[np.arange(T.shape[0]), choice]
    return (chosen - best) / best
