"""Steady-state drivers: step until the residual falls below a tolerance.

The residual is the per-step normalised change over the last K steps,
r = |u^n - u^(n-K)|_2 / (K |u^n|_2), computed in FP64 by the library's reduction
kernel; the same for phi.  A lattice (or batch instance) has converged when both
residuals are below `tol`.  Non-finite states stop the run and are reported.
"""
from __future__ import annotations

import math
import time

import numpy as np


def run_to_steady(lat, tol=1e-8, max_steps=200_000, check_every=100, log=None):
    lat.reduce(raise_nonfinite=False)          # first snapshot
    t0 = time.perf_counter()
    steps = 0
    res_u = res_phi = math.inf
    status = "max_steps"
    while steps < max_steps:
        k = min(check_every, max_steps - steps)
        lat.step(k)
        steps += k
        s = lat.reduce(raise_nonfinite=False)
        res_u, res_phi = s["res_u"], s["res_phi"]
        if s["nonfinite"] > 0:
            status = "nonfinite"
            break
        if log is not None:
            log(steps, s)
        if res_u < tol and res_phi < tol:
            status = "converged"
            break
    return {"status": status, "steps": steps, "res_u": res_u, "res_phi": res_phi,
            "seconds": time.perf_counter() - t0}


def batch_run_to_steady(batch, tol=1e-8, max_steps=200_000, check_every=100, freeze_converged=True, log=None,
                        log_every=50, max_seconds=None):
    """Steps the whole batch until every instance has converged (or gone non-finite)
    or max_steps; returns per-instance status and the step count at convergence.

    With freeze_converged, an instance leaves the step list once it has converged or
    gone non-finite (ddf_batch_set_active), so the remaining instances run alone; its
    state stays as it was at convergence.  max_seconds bounds the wall time: the run
    stops at the first check past it and unfinished instances report "max_steps"."""
    if check_every % 2 or max_steps % 2 or batch.step_count % 2:
        raise ValueError("check_every, max_steps and the batch step count must be even (active-list changes)")
    n = batch.n
    batch.reduce()
    done_at = np.full(n, -1, dtype=np.int64)
    bad = np.zeros(n, dtype=bool)
    active = np.ones(n, dtype=bool)
    t0 = time.perf_counter()
    steps = 0
    last = None
    checks = 0
    while steps < max_steps:
        k = min(check_every, max_steps - steps)
        s = batch.step_reduce(k)      # the reduction rides in the last graph replay
        steps += k
        checks += 1
        bad |= s["nonfinite"] > 0
        conv = (s["res_u"] < tol) & (s["res_phi"] < tol) & (done_at < 0) & ~bad
        done_at[conv] = steps
        if last is None:
            last = {k2: v.copy() for k2, v in s.items()}
        else:
            # frozen instances report a zero residual: keep the values they converged with
            for k2, v in s.items():
                last[k2][active] = v[active]
        finished = (done_at >= 0) | bad
        if log is not None and (checks % log_every == 0 or np.all(finished)):
            log(steps, int(np.sum(finished)), n, time.perf_counter() - t0)
        if np.all(finished) or (max_seconds is not None and time.perf_counter() - t0 > max_seconds):
            break
        if freeze_converged and np.any(active & finished) and (batch.step_count % 2 == 0):
            active &= ~finished
            batch.set_active(active)
    if freeze_converged and not np.all(active):
        batch.set_active(np.ones(n, dtype=bool))
    status = np.where(bad, "nonfinite", np.where(done_at >= 0, "converged", "max_steps"))
    return {"status": status, "steps_to_converge": done_at, "steps": steps, "stats": last,
            "seconds": time.perf_counter() - t0}
