"""GPU tests of the cavity surrogate's warm start: the trained network (weights shipped
with the package) shortens the run to r < 1e-8 at least twofold against both a cold
start and an untrained network, the warm-started steady states are the cold-started
ones (u, phi, omega within 1e-3), and the fallback re-initialises exactly the
instances whose prediction is unusable."""
import os
import sys

import numpy as np
import pytest
import torch

import workloads as W
from paper_1908_06742_amd import Batch
from paper_1908_06742_amd import surrogate as S
from paper_1908_06742_amd.steady import batch_run_to_steady

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
N = 256
WEIGHTS = os.path.join(os.path.dirname(S.__file__), "weights", "unet_cavity256.npz")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def held_out(count, lowest_re=None):
    cases = W.surrogate_cases(200, W.SURROGATE_HELDOUT_SEED0)
    idx = list(range(len(cases)))
    if lowest_re:
        idx = sorted(idx, key=lambda i: cases[i][0])[:lowest_re]
    return [cases[i] for i in idx[:count]]


def tensors(cases):
    re = torch.tensor([c[0] for c in cases], dtype=torch.float32, device=DEV)
    u = torch.tensor([c[1] for c in cases], dtype=torch.float32, device=DEV)
    return re, u


def batch_of(cases):
    return Batch([W.cavity_problem(N, re, u) for re, u in cases], device=DEV)


def cold_init(b, n):
    z = torch.zeros((n, N, N), dtype=torch.float64, device=DEV)
    b.init_device(torch.ones_like(z), z, z, z)


def cold_fields(i):
    return W.cavity_fields(N)


def steps_to(b, tol, cap):
    r = batch_run_to_steady(b, tol=tol, max_steps=cap, check_every=100)
    s = r["steps_to_converge"].astype(np.float64)
    return np.where(s >= 0, s, cap), r


def test_trained_network_shortens_the_run_to_steady_and_keeps_its_result():
    # the 8 lowest-Re held-out cavities converge to r < 1e-8 within the cap from rest
    say("case: surrogate gain, 8 lowest-Re held-out cavities, r < 1e-8")
    assert os.path.exists(WEIGHTS), "trained weights missing"
    cases = held_out(8, lowest_re=8)
    re, u = tensors(cases)
    cap = 400_000
    bc = batch_of(cases)
    cold_init(bc, len(cases))
    s_cold, rc = steps_to(bc, 1e-8, cap)
    net, meta = S.load_weights(WEIGHTS, device=DEV)
    bw = batch_of(cases)
    fb = S.warm_start_batch(net, bw, re, u, cold_fields)
    assert not fb.any()
    s_warm, rw = steps_to(bw, 1e-8, cap)
    s_warm = s_warm + 100
    untrained = S.UNet(base=32, levels=4, device=DEV, seed=0)
    bu = batch_of(cases)
    fbu = S.warm_start_batch(untrained, bu, re, u, cold_fields)
    s_untr, _ = steps_to(bu, 1e-8, cap)
    s_untr = s_untr + 100
    say(f"steps cold {s_cold.tolist()}\n      warm {s_warm.tolist()}\n untrained {s_untr.tolist()} "
        f"(fallbacks {int(fbu.sum())})")
    assert np.all(rc["status"] == "converged") and np.all(rw["status"] == "converged")
    assert s_warm.sum() * 2 <= s_cold.sum()
    assert s_warm.sum() * 2 <= s_untr.sum()
    # the lattice decides convergence: the warm-started steady state is the cold-started one
    # (both stop at r < 1e-8, so they differ by about r over the slowest decay rate)
    for i in range(len(cases)):
        a = bc.extract(i, ["ux", "uy", "phi", "wz"])
        c = bw.extract(i, ["ux", "uy", "phi", "wz"])
        m = a["phi"] >= 0.1
        du = torch.sqrt(torch.sum((a["ux"] - c["ux"]) ** 2 + (a["uy"] - c["uy"]) ** 2))
        assert float(du / torch.sqrt(torch.sum(a["ux"] ** 2 + a["uy"] ** 2))) < 1e-3, i
        assert float(torch.linalg.norm(a["phi"] - c["phi"]) / torch.linalg.norm(a["phi"])) < 1e-3, i
        e = float(torch.linalg.norm((a["wz"] - c["wz"])[m]) / torch.linalg.norm(a["wz"][m]))
        assert e < 1e-3, (i, e)


class _Scripted:
    """Wraps the trained network and spoils its prediction in chosen instances: NaN at
    one node, or a wildly wrong (Mach ~0.5) velocity field."""

    def __init__(self, net, nan_at, wild_at):
        self.net, self.device = net, net.device
        self.nan_at, self.wild_at = set(nan_at), set(wild_at)
        self.offset = 0

    def predict_fields(self, re, u, H, W):
        rho, ux, uy, phi = self.net.predict_fields(re, u, H, W)
        for j in range(re.numel()):
            g = self.offset + j
            if g in self.nan_at:
                ux[j, H // 2, W // 2] = float("nan")
            if g in self.wild_at:
                ux[j] = 0.3 * torch.sin(torch.arange(W, device=DEV, dtype=torch.float64) * 1.3)
                uy[j] = 0.3 * torch.cos(torch.arange(H, device=DEV, dtype=torch.float64)[:, None] * 0.7)
        self.offset += re.numel()
        return rho, ux, uy, phi


def test_fallback_reinitialises_exactly_the_bad_instances():
    say("case: surrogate fallback")
    cases = held_out(6)
    re, u = tensors(cases)
    net, _ = S.load_weights(WEIGHTS, device=DEV)
    b = batch_of(cases)
    fake = _Scripted(net, nan_at=[1, 4], wild_at=[2])
    fb = S.warm_start_batch(fake, b, re, u, cold_fields, chunk=4)
    assert fb.tolist() == [False, True, True, False, True, False]
    ref = batch_of(cases)
    cold_init(ref, len(cases))
    for i in range(len(cases)):
        f, g = b.get_populations(i, raw=True)
        if fb[i]:
            fr, gr = ref.get_populations(i, raw=True)
            assert torch.equal(f, fr) and torch.equal(g, gr), i
        else:
            assert torch.isfinite(f.float()).all()
    b.step(200)
    s = b.reduce()
    assert np.all(s["nonfinite"] == 0)


def test_corrupted_network_falls_back_everywhere():
    say("case: surrogate corrupted weights")
    cases = held_out(4)
    re, u = tensors(cases)
    net, _ = S.load_weights(WEIGHTS, device=DEV)
    net.w.mul_(float("nan"))
    net.cast()
    b = batch_of(cases)
    fb = S.warm_start_batch(net, b, re, u, cold_fields)
    assert fb.all()
    b.step(100)
    assert np.all(b.reduce()["nonfinite"] == 0)


def test_batch_created_while_a_prediction_is_in_flight():
    # Regression: a batch created right after a prediction whose outputs were dropped
    # receives memory the allocator recycled while the prediction's kernels may still
    # write it; the batch's setup must wait for them before uploading its tile lists.
    say("case: batch created behind in-flight prediction kernels")
    cases = held_out(16, lowest_re=16)
    re, u = tensors(cases)
    net, _ = S.load_weights(WEIGHTS, device=DEV)
    S.predict_batch_fields(net, re, u, N, N)          # outputs dropped at once
    b = batch_of(cases)
    cold_init(b, len(cases))
    b.step(200)
    s = b.reduce()
    assert np.all(s["nonfinite"] == 0)
    torch.cuda.synchronize()
    ref = batch_of(cases)
    cold_init(ref, len(cases))
    ref.step(200)
    for i in range(len(cases)):
        fa, ga = b.get_populations(i, raw=True)
        fr, gr = ref.get_populations(i, raw=True)
        assert torch.equal(fa, fr) and torch.equal(ga, gr), i
