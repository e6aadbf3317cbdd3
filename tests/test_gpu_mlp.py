"""GPU parity of the cost-model kernels (spmd_mlp.h) against the FP64 oracle,
and of the schedule-timing entry point (spmd_tune.h)."""

import numpy as np
import pytest

from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


def say(*a):
    print("case:", *a, flush=True)


@pytest.fixture(scope="module")
def L():
    import paper_2206_07896_amd as spmd  # noqa: F401  (fails loudly without the library)
    from paper_2206_07896_amd import learned

    return learned


def cuda(a, dtype=None):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype or np.float32)).cuda()


def rel_norm(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    d = np.linalg.norm(a - b)
    return d / max(np.linalg.norm(b), 1e-300)


def _problem(n, seed):
    rng = np.random.default_rng(seed)
    X = (rng.standard_normal((n, 12)) * 3.0 + 1.0).astype(np.float32)
    t = (rng.standard_normal(n) * 2.0).astype(np.float32)
    p = omlp.init_params(seed).astype(np.float32)
    p[omlp.NPARAM - 1] = 0.5
    # fixed normalisation (a one-row batch has no spread to normalise by)
    mu = np.full(12, 1.0, np.float32)
    inv_sd = np.full(12, 1.0 / 3.0, np.float32)
    return X, t, p, mu, inv_sd


def ok(rc, what):
    """Raise with the library's own message when an entry point fails."""
    import paper_2206_07896_amd as spmd

    spmd._check(rc, what)


def _fwd(L, p, norm, X, store=True):
    import torch

    n = X.shape[0]
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    h1 = torch.empty(64 * n, dtype=torch.float32, device="cuda") if store else None
    h2 = torch.empty(64 * n, dtype=torch.float32, device="cuda") if store else None
    ok(L._lib.spmd_mlp_forward(p.data_ptr(), norm.data_ptr(), X.data_ptr(), n, y.data_ptr(),
                               h1.data_ptr() if store else None, h2.data_ptr() if store else None, None),
       "spmd_mlp_forward")
    return y, h1, h2


@pytest.mark.parametrize("n", [1, 63, 64, 1000])
def test_forward_matches_oracle(L, n):
    say("mlp forward", n)
    X, t, p, mu, inv_sd = _problem(n, 100 + n)
    dp, dn, dx = cuda(p), cuda(np.concatenate([mu, inv_sd])), cuda(X)
    y, h1, h2 = _fwd(L, dp, dn, dx)
    y0, _, _ = _fwd(L, dp, dn, dx, store=False)
    yh, y0h = y.cpu().numpy(), y0.cpu().numpy()
    h1h, h2h = h1.cpu().numpy().reshape(64, n).T, h2.cpu().numpy().reshape(64, n).T
    yo, (_, _, h1o, _, h2o) = omlp.forward(p.astype(np.float64), X, mu.astype(np.float64), inv_sd.astype(np.float64))
    assert rel_norm(yh, yo) <= 1e-5
    assert np.array_equal(yh, y0h)
    assert rel_norm(h1h, h1o) <= 1e-5
    assert rel_norm(h2h, h2o) <= 1e-5


@pytest.mark.parametrize("n", [1, 64, 1000, 5000])
def test_backward_matches_oracle(L, n):
    import torch

    say("mlp backward", n)
    X, t, p, mu, inv_sd = _problem(n, 200 + n)
    dp, dn, dx, dt = cuda(p), cuda(np.concatenate([mu, inv_sd])), cuda(X), cuda(t)
    y, h1, h2 = _fwd(L, dp, dn, dx)
    ws = torch.empty(int(L._lib.spmd_mlp_workspace_size(n)), dtype=torch.uint8, device="cuda")
    g = torch.empty(omlp.NPARAM, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    for rep in range(2):  # deterministic: same bits twice
        ok(L._lib.spmd_mlp_backward(dp.data_ptr(), dn.data_ptr(), dx.data_ptr(), dt.data_ptr(), n, y.data_ptr(),
                                    h1.data_ptr(), h2.data_ptr(), g.data_ptr(), loss.data_ptr(), ws.data_ptr(),
                                    ws.numel(), None), "spmd_mlp_backward")
        gg = g.cpu().numpy()
        if rep == 0:
            first = gg.copy()
        else:
            assert np.array_equal(first, gg)
    args = (p.astype(np.float64), X, t, mu.astype(np.float64), inv_sd.astype(np.float64))
    go = omlp.unpack(omlp.grad(*args))
    gu = omlp.unpack(gg)
    for name in go:
        assert rel_norm(gu[name], go[name]) <= 1e-4, name
    lossh = float(loss.item())
    assert abs(lossh - omlp.loss(*args)) <= 1e-5 * omlp.loss(*args)


def test_backward_rejects_small_workspace(L):
    import torch

    n = 200
    X, t, p, mu, inv_sd = _problem(n, 7)
    dp, dn, dx, dt = cuda(p), cuda(np.concatenate([mu, inv_sd])), cuda(X), cuda(t)
    y, h1, h2 = _fwd(L, dp, dn, dx)
    need = int(L._lib.spmd_mlp_workspace_size(n))
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    g = torch.empty(omlp.NPARAM, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    rc = L._lib.spmd_mlp_backward(dp.data_ptr(), dn.data_ptr(), dx.data_ptr(), dt.data_ptr(), n, y.data_ptr(),
                                  h1.data_ptr(), h2.data_ptr(), g.data_ptr(), loss.data_ptr(), ws.data_ptr(),
                                  need - 4, None)
    assert rc == -8  # SPMD_ERR_WORKSPACE


@pytest.mark.parametrize("step", [1, 7, 1000])
def test_adam_matches_oracle(L, step):
    say("mlp adam", step)
    rng = np.random.default_rng(step)
    p = rng.standard_normal(omlp.NPARAM).astype(np.float32)
    g = (rng.standard_normal(omlp.NPARAM) * 0.1).astype(np.float32)
    m = (rng.standard_normal(omlp.NPARAM) * 0.05).astype(np.float32)
    v = (rng.random(omlp.NPARAM) * 0.01).astype(np.float32)
    if step == 1:
        m[:] = 0.0
        v[:] = 0.0
    dp, dg, dm, dv = cuda(p), cuda(g), cuda(m), cuda(v)
    lr = 1e-3
    ok(L._lib.spmd_mlp_adam(dp.data_ptr(), dg.data_ptr(), dm.data_ptr(), dv.data_ptr(), step, lr, 0.9, 0.999,
                            1e-8, None), "spmd_mlp_adam")
    # the entry point takes lr and the betas as fp32: the oracle gets the same values
    f32 = lambda a: float(np.float32(a))  # noqa: E731
    po, mo, vo = omlp.adam_step(p.astype(np.float64), g.astype(np.float64), m.astype(np.float64),
                                v.astype(np.float64), step, f32(lr), f32(0.9), f32(0.999), f32(1e-8))
    pg = dp.cpu().numpy().astype(np.float64)
    mg, vg = dm.cpu().numpy(), dv.cpu().numpy()
    ulp = np.spacing(np.abs(po).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(pg - po) <= 2 * ulp + 1e-5 * lr)
    # fp32 rounding of b1*m + (1-b1)*g, relative to its terms (they may cancel)
    mscale = f32(0.9) * np.abs(m.astype(np.float64)) + (1 - f32(0.9)) * np.abs(g.astype(np.float64))
    assert np.all(np.abs(mg - mo) <= 4e-7 * mscale + 1e-30)
    assert np.allclose(vg, vo, rtol=1e-6, atol=1e-14)


def _choose(L, params, norm, feats, cands, valid):
    import torch

    m, c = feats.shape[0], cands.shape[0]
    best = torch.empty(m, dtype=torch.int32, device="cuda")
    pred = torch.empty(m, dtype=torch.float32, device="cuda")
    sd = torch.empty(m, dtype=torch.float32, device="cuda")
    dp, dn, df, dc = cuda(np.concatenate(params)), cuda(norm), cuda(feats), cuda(cands)
    dv = cuda(valid.astype(np.uint8), np.uint8)
    ok(L._lib.spmd_mlp_choose(dp.data_ptr(), len(params), dn.data_ptr(), df.data_ptr(), m, dc.data_ptr(), c,
                              dv.data_ptr(), best.data_ptr(), pred.data_ptr(), sd.data_ptr(), None), "spmd_mlp_choose")
    return best.cpu().numpy().view(np.uint32), pred.cpu().numpy(), sd.cpu().numpy()


@pytest.mark.parametrize("k,c", [(1, 120), (3, 120), (4, 256), (2, 1), (3, 37)])
def test_choose_matches_oracle(L, k, c):
    say("mlp choose", k, c)
    rng = np.random.default_rng(1000 * k + c)
    m = 300
    feats = (rng.standard_normal((m, 9)) * 2.0).astype(np.float32)
    cands = (rng.standard_normal((c, 3)) * 2.0).astype(np.float32)
    valid = rng.random((m, c)) < 0.8
    valid[5, :] = False
    valid[6, :] = False
    valid[6, c - 1] = True
    params = []
    for q in range(k):
        pq = omlp.init_params(50 + q).astype(np.float32)
        pq[omlp.NPARAM - 1] = 0.3 * q
        params.append(pq)
    mu = rng.standard_normal(12).astype(np.float32) * 0.1
    inv_sd = (0.5 + rng.random(12)).astype(np.float32)
    best, pred, sd = _choose(L, params, np.concatenate([mu, inv_sd]), feats, cands, valid)
    ob, om, osd = omlp.ensemble_choose([q.astype(np.float64) for q in params], feats, cands, valid,
                                       mu.astype(np.float64), inv_sd.astype(np.float64))
    assert best[5] == 0xFFFFFFFF and ob[5] == -1
    assert best[6] == c - 1
    # the oracle's mean over every (launch, candidate), to recognise near-ties
    X = np.concatenate([np.repeat(feats, c, axis=0), np.tile(cands, (m, 1))], axis=1)
    means = np.mean([omlp.forward(q.astype(np.float64), X, mu.astype(np.float64), inv_sd.astype(np.float64))[0]
                     for q in params], axis=0).reshape(m, c)
    means = np.where(valid, means, np.inf)
    sds = np.std([omlp.forward(q.astype(np.float64), X, mu.astype(np.float64), inv_sd.astype(np.float64))[0]
                  for q in params], axis=0).reshape(m, c)
    scale = max(1.0, float(np.max(np.abs(means[np.isfinite(means)]))))
    for i in range(m):
        if ob[i] < 0:
            assert best[i] == 0xFFFFFFFF
            continue
        j = int(best[i])
        assert j < c and valid[i, j]
        # chosen candidate is optimal to within fp32 rounding of the predictions
        assert means[i, j] <= om[i] + 1e-5 * scale
        srt = np.sort(means[i][np.isfinite(means[i])])
        if srt.size == 1 or srt[1] - srt[0] > 1e-4 * scale:
            assert j == ob[i]
        assert abs(pred[i] - means[i, j]) <= 1e-5 * scale
        assert abs(sd[i] - sds[i, j]) <= 1e-5 * scale


def test_one_training_step_matches_oracle_and_training_descends(L):
    import torch

    say("mlp training step")
    n = 777
    X, _, p, mu, inv_sd = _problem(n, 31)
    t = (np.sin(X[:, 0]) + 0.1 * X[:, 1] ** 2).astype(np.float32)
    norm = np.concatenate([mu, inv_sd])
    dp, dn, dx, dt = cuda(p), cuda(norm), cuda(X), cuda(t)
    dm = torch.zeros(omlp.NPARAM, dtype=torch.float32, device="cuda")
    dv = torch.zeros_like(dm)
    ws = torch.empty(int(L._lib.spmd_mlp_workspace_size(n)), dtype=torch.uint8, device="cuda")
    g = torch.empty(omlp.NPARAM, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    losses = []
    for step in range(1, 301):
        y, h1, h2 = _fwd(L, dp, dn, dx)
        ok(L._lib.spmd_mlp_backward(dp.data_ptr(), dn.data_ptr(), dx.data_ptr(), dt.data_ptr(), n, y.data_ptr(),
                                    h1.data_ptr(), h2.data_ptr(), g.data_ptr(), loss.data_ptr(), ws.data_ptr(),
                                    ws.numel(), None), "spmd_mlp_backward")
        ok(L._lib.spmd_mlp_adam(dp.data_ptr(), g.data_ptr(), dm.data_ptr(), dv.data_ptr(), step, 3e-3, 0.9,
                                0.999, 1e-8, None), "spmd_mlp_adam")
        losses.append(float(loss.item()))
        if step == 1:
            args = (mu.astype(np.float64), inv_sd.astype(np.float64))
            go = omlp.grad(p.astype(np.float64), X, t, *args)
            po, _, _ = omlp.adam_step(p.astype(np.float64), go, np.zeros(omlp.NPARAM), np.zeros(omlp.NPARAM), 1,
                                      3e-3)
            # the first step is lr * sign(g): compare where the sign is not decided by rounding
            big = np.abs(go) > 1e-3 * np.sqrt(np.mean(go * go))
            dg = dp.cpu().numpy().astype(np.float64) - p
            assert rel_norm(dg[big], (po - p)[big]) <= 1e-4
    assert losses[-1] < 0.2 * losses[0]


def test_tune_time_measures_and_computes(L):
    import torch

    import paper_2206_07896_amd as spmd
    import synth

    say("tune time reduce")
    n = 300_001
    x = synth.uniform_int32(0x7E, n, -1000, 1000)
    tin = cuda(x, np.int32)
    tout = torch.zeros(1, dtype=torch.int32, device="cuda")
    tuner = L.Autotuner(reps=2)
    scheds = [(64, 1, 1), (256, 4, 8), (512, 16, 32)]
    ms = tuner.time((spmd.REDUCE_I32, n, 1, 256, tin, tout), scheds)
    total = int(tout.item())
    assert ms.shape == (3,) and np.all(np.isfinite(ms)) and np.all(ms > 0)
    assert total == int(x.astype(np.int64).sum())  # closed form, |sum| < 2^31
    with pytest.raises(ValueError):
        tuner.time((spmd.REDUCE_I32, n, 1, 256, tin, tout), [(256, 3, 1)])


def test_contention_study_rows(L):
    """The skewed-key schedule study: one row per key distribution, the
    regrets are ratios of timings of the same instance (>= 0), and the
    exponent-1.1 row's own best has zero regret."""
    say("contention study 2^12")
    rows = L.contention_study(None, log2_sizes=(12,), reps=1)
    assert [r["keys"] for r in rows] == ["zipf0", "zipf1.1", "zipf2", "zipf3", "one bin"]
    cands = {tuple(c) for c in L.CANDIDATES}
    for r in rows:
        assert r["log2_n"] == 12 and r["best_us"] > 0 and tuple(r["best"]) in cands
        assert r["regret_of_zipf1.1_best"] >= 0
    assert rows[1]["regret_of_zipf1.1_best"] == 0


@pytest.mark.parametrize("slack", [0.0, 0.05, 0.2, 1.0])
def test_choose_batch_matches_oracle(L, slack):
    """spmd_mlp_choose_batch against the FP64 oracle's batch-aware rule:
    fewest chunks among the candidates within ln(1 + slack) of the least
    mean.  Launches with a candidate within fp32 rounding of the threshold
    are checked for validity only."""
    import torch

    say("mlp choose batch", slack)
    rng = np.random.default_rng(77)
    m, c, k = 200, 120, 3
    feats = (rng.standard_normal((m, 9)) * 2.0).astype(np.float32)
    cands = (rng.standard_normal((c, 3)) * 2.0).astype(np.float32)
    valid = rng.random((m, c)) < 0.8
    valid[3, :] = False
    chunks = rng.integers(1, 40, (m, c)).astype(np.uint32)
    params = [omlp.init_params(60 + q).astype(np.float32) for q in range(k)]
    mu = rng.standard_normal(12).astype(np.float32) * 0.1
    inv_sd = (0.5 + rng.random(12)).astype(np.float32)
    best = torch.empty(m, dtype=torch.int32, device="cuda")
    pred = torch.empty(m, dtype=torch.float32, device="cuda")
    sd = torch.empty(m, dtype=torch.float32, device="cuda")
    dp, dn, df, dc = cuda(np.concatenate(params)), cuda(np.concatenate([mu, inv_sd])), cuda(feats), cuda(cands)
    dv = cuda(valid.astype(np.uint8), np.uint8)
    dch = cuda(chunks.view(np.int32), np.int32)
    ok(L._lib.spmd_mlp_choose_batch(dp.data_ptr(), k, dn.data_ptr(), df.data_ptr(), m, dc.data_ptr(), c,
                                    dv.data_ptr(), dch.data_ptr(), float(slack), best.data_ptr(), pred.data_ptr(),
                                    sd.data_ptr(), None), "spmd_mlp_choose_batch")
    got = best.cpu().numpy().view(np.uint32)
    p64 = [q.astype(np.float64) for q in params]
    ob, om, osd = omlp.ensemble_choose_batch(p64, feats, cands, valid, chunks, slack, mu.astype(np.float64),
                                             inv_sd.astype(np.float64))
    X = np.concatenate([np.repeat(feats, c, axis=0), np.tile(cands, (m, 1))], axis=1)
    means = np.mean([omlp.forward(q, X, mu.astype(np.float64), inv_sd.astype(np.float64))[0] for q in p64],
                    axis=0).reshape(m, c)
    means = np.where(valid, means, np.inf)
    scale = max(1.0, float(np.max(np.abs(means[np.isfinite(means)]))))
    tol = 1e-4 * scale
    assert got[3] == 0xFFFFFFFF and ob[3] == -1
    strict = 0
    for i in range(m):
        if ob[i] < 0:
            continue
        j = int(got[i])
        assert j < c and valid[i, j]
        thr = np.min(means[i]) + np.log1p(slack)
        assert means[i, j] <= thr + tol
        inside = means[i] <= thr - tol
        if inside.any():  # candidates surely within the slack: none has fewer chunks
            assert chunks[i, j] <= chunks[i][inside].min()
        boundary = np.abs(means[i] - thr) <= tol
        if slack == 0:
            boundary[np.argmin(means[i])] = False  # at slack 0 the least itself sits on the threshold
        if not boundary.any():
            ties = np.sort(means[i][(chunks[i] == chunks[i, j]) & (means[i] <= thr)])
            if ties.size == 1 or ties[1] - ties[0] > tol:
                assert j == ob[i], i
                strict += 1
    assert strict > m // 2
