"""FP64 reference of the schedule cost model.  TEST INFRASTRUCTURE ONLY.

A two-hidden-layer perceptron predicting the log running time of a launch
under a candidate schedule:

    z1 = xn W1 + b1,  h1 = relu(z1)          xn = (x - mu) * inv_sd
    z2 = h1 W2 + b2,  h2 = relu(z2)
    y  = h2 . w3 + b3

trained on the mean squared error mean((y - t)^2) with Adam (Kingma and Ba,
"Adam: A Method for Stochastic Optimization", 2015).  relu'(0) is taken as
0.  Parameters live in one flat vector in the order W1 (DIN x H, row-major),
b1, W2 (H x H), b2, w3, b3 -- the layout the GPU kernels use.
"""

from __future__ import annotations

import numpy as np

DIN = 12
H = 64
SIZES = [("W1", (DIN, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("w3", (H,)), ("b3", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(p):
    out, o = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = np.asarray(p[o:o + k], dtype=np.float64).reshape(shape)
        o += k
    return out


def pack(d) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in SIZES])


def forward(p, X, mu=None, inv_sd=None):
    """Predictions y[N] and the intermediate activations."""
    w = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    xn = X if mu is None else (X - mu) * inv_sd
    z1 = xn @ w["W1"] + w["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ w["W2"] + w["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w["w3"] + w["b3"][0]
    return y, (xn, z1, h1, z2, h2)


def loss(p, X, t, mu=None, inv_sd=None) -> float:
    y, _ = forward(p, X, mu, inv_sd)
    return float(np.mean((y - np.asarray(t, dtype=np.float64)) ** 2))


def grad(p, X, t, mu=None, inv_sd=None):
    """Analytic gradient of `loss` with respect to the flat parameters."""
    w = unpack(p)
    y, (xn, z1, h1, z2, h2) = forward(p, X, mu, inv_sd)
    n = y.shape[0]
    dy = 2.0 * (y - np.asarray(t, dtype=np.float64)) / n
    g = {"w3": h2.T @ dy, "b3": np.array([dy.sum()])}
    dz2 = np.outer(dy, w["w3"]) * (z2 > 0)
    g["W2"] = h1.T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ w["W2"].T) * (z1 > 0)
    g["W1"] = xn.T @ dz1
    g["b1"] = dz1.sum(axis=0)
    return pack(g)


def adam_step(p, g, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update (step counts from 1); returns new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def init_params(seed: int, scale1: float = None, scale2: float = None) -> np.ndarray:
    """He-style initial weights from a seeded generator (biases zero)."""
    rng = np.random.default_rng(seed)
    d = {
        "W1": rng.standard_normal((DIN, H)) * (scale1 if scale1 else np.sqrt(2.0 / DIN)),
        "b1": np.zeros(H),
        "W2": rng.standard_normal((H, H)) * (scale2 if scale2 else np.sqrt(2.0 / H)),
        "b2": np.zeros(H),
        "w3": rng.standard_normal(H) * np.sqrt(1.0 / H),
        "b3": np.zeros(1),
    }
    return pack(d)


def ensemble_choose(params_list, feats, cands, valid, mu=None, inv_sd=None):
    """Schedule choice of an ensemble: for each launch (row of feats) every
    valid candidate (row of cands) is scored by the mean prediction of the
    models; the chosen index minimises it (the lowest index among equal
    means).  Returns (index, mean there, population standard deviation of
    the models' predictions there); index -1 when no candidate is valid."""
    feats = np.asarray(feats, dtype=np.float64)
    cands = np.asarray(cands, dtype=np.float64)
    m, c = feats.shape[0], cands.shape[0]
    best = np.full(m, -1, dtype=np.int64)
    mean_at = np.full(m, np.inf)
    sd_at = np.zeros(m)
    for i in range(m):
        X = np.concatenate([np.repeat(feats[i:i + 1], c, axis=0), cands], axis=1)
        preds = np.stack([forward(p, X, mu, inv_sd)[0] for p in params_list])
        mean = preds.mean(axis=0)
        sd = preds.std(axis=0)
        for j in range(c):
            if valid[i][j] and (best[i] < 0 or mean[j] < mean_at[i]):
                best[i], mean_at[i], sd_at[i] = j, mean[j], sd[j]
    return best, mean_at, sd_at


def ensemble_choose_batch(params_list, feats, cands, valid, chunks, slack, mu=None, inv_sd=None):
    """Batch-aware choice (not in the paper; the library's rule for a batch,
    where every chunk is one fetch from a shared cursor): per launch, the
    valid candidates whose mean prediction is at most the least mean plus
    ln(1 + slack); among them the fewest chunks, then the smaller mean, then
    the lower index.  Returns (index, mean there, sd there); -1 when no
    candidate is valid."""
    feats = np.asarray(feats, dtype=np.float64)
    cands = np.asarray(cands, dtype=np.float64)
    m, c = feats.shape[0], cands.shape[0]
    best = np.full(m, -1, dtype=np.int64)
    mean_at = np.full(m, np.inf)
    sd_at = np.zeros(m)
    for i in range(m):
        X = np.concatenate([np.repeat(feats[i:i + 1], c, axis=0), cands], axis=1)
        preds = np.stack([forward(p, X, mu, inv_sd)[0] for p in params_list])
        mean = preds.mean(axis=0)
        sd = preds.std(axis=0)
        ok = [j for j in range(c) if valid[i][j]]
        if not ok:
            continue
        least = min(mean[j] for j in ok)
        near = [j for j in ok if mean[j] <= least + np.log1p(slack)]
        j = min(near, key=lambda q: (int(chunks[i][q]), mean[q], q))
        best[i], mean_at[i], sd_at[i] = j, mean[j], sd[j]
    return best, mean_at, sd_at
