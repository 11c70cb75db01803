"""Host-side checks of the run-to-steady driver (no GPU): a scripted batch whose
instances' residuals fall at known rates."""
import numpy as np
import pytest

from paper_1908_06742_amd.steady import batch_run_to_steady


class ScriptedBatch:
    """Instance i's residual is r0 * exp(-rate_i * step) while it steps; a frozen
    instance's residual reads 0 (it does not change), like the library's batch."""

    def __init__(self, rates, r0=1e-2, nonfinite_at=None):
        self.rates = np.asarray(rates, float)
        self.n = len(rates)
        self.r0 = r0
        self.step_count = 0
        self.active = np.ones(self.n, bool)
        self.age = np.zeros(self.n)
        self.active_calls = []
        self.nonfinite_at = nonfinite_at or {}

    def step(self, k):
        self.step_count += k
        self.age[self.active] += k
        return self

    def reduce(self, raise_nonfinite=False):
        r = self.r0 * np.exp(-self.rates * self.age)
        r[~self.active] = 0.0
        nf = np.array([1.0 if self.step_count >= self.nonfinite_at.get(i, np.inf) else 0.0 for i in range(self.n)])
        return {"res_u": r.copy(), "res_phi": 0.5 * r, "nonfinite": nf, "mass": np.ones(self.n)}

    def step_reduce(self, k, raise_nonfinite=False):
        return self.step(k).reduce(raise_nonfinite)

    def set_active(self, active):
        if self.step_count % 2:
            raise RuntimeError("odd step count")
        self.active = np.asarray(active, bool).copy()
        self.active_calls.append(self.active.copy())


def expected_steps(rate, tol, r0, check):
    k = check
    while r0 * np.exp(-rate * k) >= tol:
        k += check
    return k


def test_instances_stop_when_converged_and_the_rest_continue():
    rates = [1e-3, 2e-4, 5e-4]
    b = ScriptedBatch(rates)
    r = batch_run_to_steady(b, tol=1e-6, max_steps=100_000, check_every=100)
    for i, rate in enumerate(rates):
        assert r["steps_to_converge"][i] == expected_steps(rate, 1e-6, 1e-2, 100)
    assert list(r["status"]) == ["converged"] * 3
    assert r["steps"] == max(r["steps_to_converge"])
    # the fastest instance left the step list first; all were re-activated at the end
    assert b.active_calls[0].tolist() == [False, True, True]
    assert b.active.all()
    # the reported residual of a frozen instance is the one it converged with, not 0
    assert 0 < r["stats"]["res_u"][0] < 1e-6


def test_cap_nonfinite_and_time_bound():
    b = ScriptedBatch([1e-2, 1e-6, 1e-3], nonfinite_at={2: 300})
    r = batch_run_to_steady(b, tol=1e-6, max_steps=2000, check_every=100)
    assert list(r["status"]) == ["converged", "max_steps", "nonfinite"]
    assert r["steps_to_converge"][1] == -1 and r["steps"] == 2000
    b = ScriptedBatch([1e-9])
    r = batch_run_to_steady(b, tol=1e-6, max_steps=10**9, check_every=100, max_seconds=0.0)
    assert r["steps"] == 100 and r["status"][0] == "max_steps"


def test_even_step_counts_are_required():
    with pytest.raises(ValueError):
        batch_run_to_steady(ScriptedBatch([1e-3]), check_every=101)
    with pytest.raises(ValueError):
        batch_run_to_steady(ScriptedBatch([1e-3]), max_steps=1001)
    b = ScriptedBatch([1e-3])
    b.step_count = 1
    with pytest.raises(ValueError):
        batch_run_to_steady(b)
