"""The learned schedule end to end on the GPU, at a small scale: exhaustive
tuning of launches drawn like the mixed workload, training of the ensemble
by the library's kernels, and the choice on held-out launches scored against
their own exhaustive timings.  What the model gains over the method without
it (the paper's as-launched schedule with average coarse-grained fetching)
is the ratio of their summed times on the held-out launches."""

import math

import pytest

pytestmark = pytest.mark.gpu


def test_learned_schedule_beats_heuristic_small():
    import paper_2206_07896_amd  # noqa: F401  (fails loudly without the library)
    from paper_2206_07896_amd import learned as L

    print("case: learned schedule, 64 train / 64 held-out launches, n <= 2^16", flush=True)
    res, model = L.evaluate(train_count=64, heldout_count=64, k_models=2, steps=600, reps=2, batch_reps=3,
                            log=lambda m: print(m, flush=True), log2_hi=16.0)
    # training by the GPU kernels lowers the loss
    for a, b in zip(res["initial_train_mse"], res["final_train_mse"]):
        assert math.isfinite(b) and b < 0.5 * a
    # the exhaustive fallback can only remove regret
    assert 0.0 <= res["regret_mean_with_fallback"] <= res["regret_mean"] + 1e-12
    assert 0.0 <= res["fallback_rate"] <= 1.0
    # the learned choice costs less in total than the paper's heuristic
    assert res["time_sum_ratio_heuristic_over_learned"] > 1.0
    assert res["regret_mean_with_fallback"] < res["regret_mean_heuristic"]


def test_shipped_model_regret_within_bound():
    """The shipped cost model on 150 held-out launches drawn like the mixed
    workload (sizes up to 2^22), each timed here under every candidate
    schedule: the mean regret of its choice, with the exhaustive fallback
    for low-confidence launches, is at most 10%."""
    import paper_2206_07896_amd  # noqa: F401
    from paper_2206_07896_amd import learned as L

    model = L.load_default()
    assert model is not None, "the package ships a cost model"
    print("case: shipped model, 150 held-out launches x every schedule", flush=True)
    res = L.heldout_regret(model, 150)
    print(res, flush=True)
    assert 0.0 <= res["regret_mean_with_fallback"] <= res["regret_mean"] + 1e-12
    assert res["regret_mean_with_fallback"] <= 0.10
    assert res["regret_mean_with_fallback"] < res["regret_mean_heuristic"]
