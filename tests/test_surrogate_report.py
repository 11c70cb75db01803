"""Host-side checks of the surrogate study's bookkeeping (no GPU): the report's
speedups and counts from hand-made arm records, and the held-out seeds being
disjoint from the training seeds."""
import pytest

import workloads as W

torch = pytest.importorskip("torch")
from paper_1908_06742_amd.surrogate_study import report  # noqa: E402


def test_report_counts_and_speedups():
    cold = {"cap": 1000, "tol": 1e-8, "n_eval": 3, "single_seconds_per_step": 0.01,
            "cold_batch": {"seconds": 5.0, "steps": [200, -1, 600], "status": ["converged", "max_steps", "converged"]}}
    warm = {"warm_batch": {"seconds": 2.5, "fallbacks": 1, "steps": [100, 700, -1],
                           "status": ["converged", "converged", "max_steps"]},
            "omega_vs_f64": [{"err": 2e-4}, {"err": 5e-4}]}
    r = report(cold, warm)
    # cold single: (200 + 1000 (capped) + 600) steps at 10 ms
    assert r["seconds_cold_single"] == pytest.approx(18.0)
    assert r["speedup_warm_batch_vs_cold_single"] == pytest.approx(18.0 / 2.5)
    assert r["speedup_warm_batch_vs_cold_batch"] == pytest.approx(2.0)
    assert (r["converged_cold"], r["converged_warm"], r["converged_both"]) == (2, 2, 1)
    assert r["median_steps_cold_over_warm"] == pytest.approx(2.0)
    assert r["omega_vs_f64_max"] == pytest.approx(5e-4)
    assert r["fallbacks"] == 1


def test_held_out_cases_are_disjoint_and_in_range():
    train = W.surrogate_cases(300, W.SURROGATE_TRAIN_SEED0)
    held = W.surrogate_cases(200, W.SURROGATE_HELDOUT_SEED0)
    assert not set(train) & set(held)
    for re, u in train + held:
        assert 100.0 <= re <= 5000.0 and 0.05 <= u <= 0.1
