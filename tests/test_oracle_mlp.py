"""Pins of the FP64 cost-model oracle: central finite differences of the
loss, special cases with known gradients, and Adam's first step."""

import numpy as np
import pytest

from oracle import mlp


def _data(n=37, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, mlp.DIN))
    t = rng.standard_normal(n)
    return X, t


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradient_matches_central_differences(seed):
    X, t = _data(seed=seed)
    mu = X.mean(axis=0)
    inv_sd = 1.0 / (X.std(axis=0) + 0.5)
    p = mlp.init_params(seed)
    p[mlp.NPARAM - 1] = 0.3
    g = mlp.grad(p, X, t, mu, inv_sd)
    rng = np.random.default_rng(seed + 10)
    idx = rng.choice(mlp.NPARAM, 200, replace=False)
    h = 1e-6
    fd = np.empty(idx.size)
    for k, i in enumerate(idx):
        e = np.zeros(mlp.NPARAM)
        e[i] = h
        fd[k] = (mlp.loss(p + e, X, t, mu, inv_sd) - mlp.loss(p - e, X, t, mu, inv_sd)) / (2 * h)
    # kinks of relu are measure-zero for random data; compare normwise
    assert np.linalg.norm(fd - g[idx]) <= 1e-6 * np.linalg.norm(g[idx])


def test_zero_weights_output_is_bias_and_only_b3_learns():
    X, t = _data()
    p = np.zeros(mlp.NPARAM)
    p[-1] = 1.25
    y, _ = mlp.forward(p, X)
    assert np.all(y == 1.25)
    g = mlp.grad(p, X, t)
    # every hidden unit is dead (z = 0, relu' = 0): only b3 has a gradient
    assert np.all(g[:-1] == 0.0)
    assert g[-1] == pytest.approx(2.0 * np.mean(1.25 - t), rel=1e-14)


def test_dead_first_layer_unit_has_zero_gradient():
    X, t = _data()
    d = mlp.unpack(mlp.init_params(3))
    d["b1"][5] = -1e6  # unit 5 of layer 1 is never active
    g = mlp.unpack(mlp.grad(mlp.pack(d), X, t))
    assert np.all(g["W1"][:, 5] == 0.0) and g["b1"][5] == 0.0
    assert np.all(g["W2"][5, :] == 0.0)


def test_linear_regime_matches_least_squares_gradient():
    # with every unit active and W2 = I, the model is affine in xn: y = xn A + c
    X, t = _data(n=50, seed=4)
    d = mlp.unpack(np.zeros(mlp.NPARAM))
    rng = np.random.default_rng(5)
    d["W1"] = rng.standard_normal((mlp.DIN, mlp.H)) * 0.01
    d["b1"][:] = 100.0
    d["W2"] = np.eye(mlp.H)
    d["w3"] = rng.standard_normal(mlp.H)
    p = mlp.pack(d)
    y, _ = mlp.forward(p, X)
    A = d["W1"] @ d["w3"]
    c = d["b1"] @ d["w3"]
    assert np.allclose(y, X @ A + c, rtol=1e-12, atol=1e-9)
    # d loss / d b3 = mean(2 (y - t))
    assert mlp.grad(p, X, t)[-1] == pytest.approx(np.mean(2 * (y - t)), rel=1e-12)


def test_adam_first_step_is_lr_times_sign():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    m = np.zeros(3)
    v = np.zeros(3)
    p1, m1, v1 = mlp.adam_step(p, g, m, v, 1, 0.01, eps=0.0)
    # bias-corrected first moments equal g and |g|: the step is lr * sign(g)
    assert np.allclose(p1, p - 0.01 * np.sign(g), rtol=0, atol=1e-15)
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)


def test_training_reduces_loss():
    X, _ = _data(n=256, seed=7)
    t = np.sin(X[:, 0]) + 0.5 * X[:, 1] ** 2
    p = mlp.init_params(1)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    l0 = mlp.loss(p, X, t)
    for s in range(1, 301):
        p, m, v = mlp.adam_step(p, mlp.grad(p, X, t), m, v, s, 3e-3)
    assert mlp.loss(p, X, t) < 0.2 * l0


def test_ensemble_choose_special_cases():
    rng = np.random.default_rng(11)
    feats = rng.standard_normal((5, 9))
    cands = rng.standard_normal((7, 3))
    valid = np.ones((5, 7), bool)
    valid[1, :3] = False
    valid[2, :] = False
    # constant models: every candidate ties, the first valid index wins
    const = np.zeros(mlp.NPARAM)
    const[-1] = 2.0
    best, mean, sd = mlp.ensemble_choose([const, const], feats, cands, valid)
    assert list(best) == [0, 3, -1, 0, 0]
    assert mean[0] == 2.0 and sd[0] == 0.0
    # one model: the choice is the argmin of its own predictions over the valid set
    p = mlp.init_params(4)
    best, mean, sd = mlp.ensemble_choose([p], feats, cands, valid)
    for i in (0, 1, 3, 4):
        y, _ = mlp.forward(p, np.concatenate([np.repeat(feats[i:i + 1], 7, 0), cands], 1))
        y = np.where(valid[i], y, np.inf)
        assert best[i] == int(np.argmin(y)) and mean[i] == y[best[i]] and sd[i] == 0.0


def test_ensemble_choose_mean_and_sd_of_two_models():
    # two models that differ only in b3 by +-d: mean is the shared part, sd = d
    rng = np.random.default_rng(12)
    feats = rng.standard_normal((3, 9))
    cands = rng.standard_normal((4, 3))
    p = mlp.init_params(5)
    a, b = p.copy(), p.copy()
    a[-1] += 0.75
    b[-1] -= 0.75
    best, mean, sd = mlp.ensemble_choose([a, b], feats, cands, np.ones((3, 4), bool))
    best1, mean1, _ = mlp.ensemble_choose([p], feats, cands, np.ones((3, 4), bool))
    assert list(best) == list(best1)
    assert np.allclose(mean, mean1, rtol=0, atol=1e-12) and np.allclose(sd, 0.75, rtol=0, atol=1e-12)


def _pass_through_model():
    """A model whose prediction is the first schedule input (x[9]) for
    x[9] >= 0: one ReLU path with unit weights, everything else zero."""
    flat = np.zeros(mlp.NPARAM)
    o = 0
    for name, shape in mlp.SIZES:
        k = int(np.prod(shape))
        if name == "W1":
            w = np.zeros(shape)
            w[9, 0] = 1.0
            flat[o:o + k] = w.ravel()
        elif name == "W2":
            w = np.zeros(shape)
            w[0, 0] = 1.0
            flat[o:o + k] = w.ravel()
        elif name == "w3":
            w = np.zeros(shape)
            w[0] = 1.0
            flat[o:o + k] = w
        o += k
    return flat


def test_ensemble_choose_batch_hand_case():
    # predictions 0, 0.1, 0.3, 0.05 (the first schedule input); chunks 10, 5, 1, 7
    p = _pass_through_model()
    feats = np.zeros((1, 9))
    cands = np.array([[0.0, 0, 0], [0.1, 0, 0], [0.3, 0, 0], [0.05, 0, 0]])
    valid = np.ones((1, 4), bool)
    chunks = np.array([[10, 5, 1, 7]])
    mu, inv_sd = np.zeros(12), np.ones(12)
    pick = lambda slack: int(mlp.ensemble_choose_batch([p], feats, cands, valid, chunks, slack, mu, inv_sd)[0][0])  # noqa: E731
    assert pick(0.0) == 0                     # nothing within slack but the least itself
    assert pick(np.expm1(0.15)) == 1          # 0, 0.1 and 0.05 are near: 5 chunks is fewest
    assert pick(np.expm1(0.35)) == 2          # all near: the single chunk wins
    assert pick(np.expm1(0.07)) == 3          # 0 and 0.05 near: 7 chunks beat 10
    valid[0, 2] = False
    assert pick(np.expm1(0.35)) == 1          # the invalid candidate is never chosen


def test_ensemble_choose_batch_reduces_to_plain_choice_and_breaks_ties():
    rng = np.random.default_rng(11)
    params = [mlp.init_params(3), mlp.init_params(4)]
    feats = rng.standard_normal((6, 9))
    cands = rng.standard_normal((20, 3))
    valid = rng.random((6, 20)) < 0.7
    chunks = rng.integers(1, 50, (6, 20))
    b0, m0, _ = mlp.ensemble_choose(params, feats, cands, valid)
    b1, m1, _ = mlp.ensemble_choose_batch(params, feats, cands, valid, chunks, 0.0)
    assert np.array_equal(b0, b1) and np.allclose(m0, m1)
    # equal predictions everywhere (zero weights, one bias): fewest chunks, then lowest index
    const = np.zeros(mlp.NPARAM)
    const[-1] = 2.5
    chunks = np.array([[4, 2, 2, 9]])
    b, m, _ = mlp.ensemble_choose_batch([const], np.zeros((1, 9)), np.zeros((4, 3)), np.ones((1, 4), bool), chunks, 0.0)
    assert int(b[0]) == 1 and m[0] == 2.5
