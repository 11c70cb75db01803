"""Cavity surrogate: training data from the solver, GPU training, and the
time-to-steady study of warm against cold starts.

    python -m paper_1908_06742_amd.surrogate_study train --n-train 512 --out unet.npz
    python -m paper_1908_06742_amd.surrogate_study cold --out cold.json
    python -m paper_1908_06742_amd.surrogate_study warm --weights unet.npz --out warm.json
    python -m paper_1908_06742_amd.surrogate_study report cold.json warm.json

Training data: 256^2 lid-driven cavities (Re log-uniform in [100, 5000], lid speed
U ~ U(0.05, 0.1), lid phi = 1, other walls phi = 0, tau_phi = tau) run in one batch until
both residuals are below 1e-8 or a step cap, converged instances leaving the step list;
from rest, or (--warm-data) from an earlier network's prediction with the same fallback
as the warm arm.  Targets are (u / U, v / U, (rho - 1) / U^2, phi) of the final states.

Evaluation on held-out seeds, each arm to r < 1e-8 (or the cap):
  cold_single  one FP32 lattice at a time: the measured per-step time of a single
               256^2 lattice (checks every 100 steps included) times each instance's
               cold step count;
  cold_batch   every instance in one batch from rest (measured wall time);
  warm_batch   network prediction, equilibrium initialisation, fallback check after
               100 steps, then the batch run (measured wall time, inference included).
The warm arm also compares omega of its steady states (normwise over nodes with
phi >= 0.1) with FP64 steady states, for converged held-out cases spread over the Re
range: the FP64 path continues each warm FP32 steady state until r < 1e-10.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

import workloads as W

from .batch import Batch
from .lattice import Lattice
from .steady import batch_run_to_steady, run_to_steady
from . import surrogate as S

N_SIDE = 256


def say(*a):
    print(*a, flush=True)


def _problems(cases, n, storage="f32"):
    return [W.cavity_problem(n, re, u, storage=storage) for re, u in cases]


def _cold(n):
    f = W.cavity_fields(n)
    return lambda i: f


def _init_cold(b, N, n, device):
    """Rest state of N cavities (rho = 1, u = 0, phi = 0) from device fields."""
    z = torch.zeros((N, n, n), dtype=torch.float64, device=device)
    b.init_device(torch.ones_like(z), z, z, z)


def _progress(tag):
    def log(steps, done, n, secs):
        say(f"  [{tag}] steps {steps:8d}  finished {done:4d}/{n}  {secs:7.1f} s")
    return log


def generate(cases, n=N_SIDE, tol=1e-8, cap=400_000, check_every=100, device="cuda", max_seconds=None, warm_net=None):
    """Runs every case to its steady state, from rest or (warm_net) from that network's
    prediction with the fallback to rest of warm_start_batch; returns FP64 device fields
    [N, n, n] (rho, ux, uy, phi) and the run record.  The solver decides convergence
    either way: the targets are lattice Boltzmann steady states."""
    b = Batch(_problems(cases, n), device=device)
    b.autotune(10)
    fb = None
    if warm_net is None:
        _init_cold(b, len(cases), n, device)
        r = batch_run_to_steady(b, tol=tol, max_steps=cap, check_every=check_every, log=_progress("data"),
                                max_seconds=max_seconds)
    else:
        re = torch.tensor([c[0] for c in cases], dtype=torch.float32, device=device)
        u = torch.tensor([c[1] for c in cases], dtype=torch.float32, device=device)
        t0 = time.perf_counter()
        fb = S.warm_start_batch(warm_net, b, re, u, _cold(n), check_steps=100, fallback_tol=1e-2)
        left = None if max_seconds is None else max(1.0, max_seconds - (time.perf_counter() - t0))
        r = batch_run_to_steady(b, tol=tol, max_steps=cap - 100, check_every=check_every, log=_progress("data"),
                                max_seconds=left)
        r["steps_to_converge"] = np.where(r["steps_to_converge"] >= 0, r["steps_to_converge"] + 100, -1)
        r["steps"] += 100
    r["fallbacks"] = None if fb is None else int(fb.sum())
    N = len(cases)
    fields = [torch.empty((N, n, n), dtype=torch.float64, device=device) for _ in range(4)]
    for i in range(N):
        e = b.extract(i, ["rho", "ux", "uy", "phi"])
        for k, nm in enumerate(("rho", "ux", "uy", "phi")):
            fields[k][i].copy_(e[nm])
    del b
    return fields, r


def cmd_train(a):
    torch.manual_seed(0)
    dev = "cuda"
    cases = W.surrogate_cases(a.n_train, W.SURROGATE_TRAIN_SEED0)
    t0 = time.perf_counter()
    warm = None
    if a.warm_data:
        warm, _ = S.load_weights(a.warm_data, device=dev)
    say(f"generating {a.n_train} steady cavities at {a.n}^2 (cap {a.cap} steps, "
        f"{'warm-started from ' + a.warm_data if warm is not None else 'from rest'})")
    fields, run = generate(cases, a.n, cap=a.cap, max_seconds=a.data_seconds, warm_net=warm)
    del warm
    t_gen = time.perf_counter() - t0
    conv = int(np.sum(run["status"] == "converged"))
    say(f"data: {t_gen:.1f} s, converged {conv}/{a.n_train}, batch steps {run['steps']}")
    res = np.maximum(run["stats"]["res_u"], run["stats"]["res_phi"])
    for q in (0.5, 0.9, 1.0):
        say(f"  final residual quantile {q}: {np.quantile(res, q):.2e}")
    re = torch.tensor([c[0] for c in cases], dtype=torch.float32, device=dev)
    u = torch.tensor([c[1] for c in cases], dtype=torch.float32, device=dev)
    targets = S.make_targets(*fields, u)
    del fields
    torch.cuda.synchronize()
    nval = max(1, a.n_train // 16)
    ntr = a.n_train - nval
    net = S.UNet(base=32, levels=4, device=dev, seed=a.seed)
    hw4 = a.n * a.n * 4
    tr_t = targets[:ntr * hw4]
    va_t = targets[ntr * hw4:]
    say(f"training: {ntr} samples, {nval} validation, {a.iters} iterations of batch {a.batch}")
    t1 = time.perf_counter()

    def log(it, loss, lr):
        say(f"  it {it:6d}  loss/pixel {loss:.4e}  lr {lr:.2e}  {time.perf_counter() - t1:7.1f} s")
    hist = S.train(net, re[:ntr], u[:ntr], tr_t, a.n, a.n, a.iters, batch_size=a.batch, lr=a.lr, log=log,
                   log_every=max(1, a.iters // 40))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    val = S.evaluate_loss(net, re[ntr:], u[ntr:], va_t, a.n, a.n)
    trn = S.evaluate_loss(net, re[:min(ntr, 64)], u[:min(ntr, 64)], tr_t[:min(ntr, 64) * hw4], a.n, a.n)
    say(f"train loss/pixel {trn:.4e}  validation loss/pixel {val:.4e}  training {t_train:.1f} s")
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    S.save_weights(net, a.out, n_train=ntr, n_val=nval, cap=a.cap, iters=a.iters, batch=a.batch, lr=a.lr,
                   val_loss=val, train_loss=trn, side=a.n, converged=conv,
                   seconds_data=t_gen, seconds_train=t_train)
    rec = {"n_train": ntr, "n_val": nval, "cap": a.cap, "converged": conv, "seconds_data": t_gen,
           "data_warm_start": a.warm_data, "data_fallbacks": run["fallbacks"],
           "data_steps": run["steps"], "data_res_u": run["stats"]["res_u"].tolist(),
           "data_res_phi": run["stats"]["res_phi"].tolist(), "data_steps_to_converge": run["steps_to_converge"].tolist(),
           "seconds_train": t_train, "ms_per_iter": 1e3 * t_train / a.iters, "val_loss": val, "train_loss": trn,
           "history": hist}
    with open(os.path.splitext(a.out)[0] + "_train.json", "w") as f:
        json.dump(rec, f, indent=1)
    say("saved", a.out)


def single_step_seconds(case, n, steps=20_000, check_every=100):
    """Per-step wall time of one FP32 n^2 cavity stepped alone, with the residual check
    every check_every steps, after a warm-up."""
    lat = Lattice(W.cavity_problem(n, *case), device="cuda").init(*W.cavity_fields(n))
    lat.step(2000)
    lat.reduce(raise_nonfinite=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps // check_every):
        lat.step(check_every)
        lat.reduce(raise_nonfinite=False)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def cmd_cold(a):
    """Cold arms: the batch from rest, and the per-step time of a single lattice."""
    dev = "cuda"
    n = a.n
    cases = W.surrogate_cases(a.n_eval, W.SURROGATE_HELDOUT_SEED0)
    N = len(cases)
    rec = {"arm": "cold", "n_eval": N, "side": n, "cap": a.cap, "tol": a.tol, "cases": cases}
    probe = Batch(_problems(cases, n), device=dev)
    rec["tiling"] = probe.autotune(10)
    del probe
    say(f"cold batch: {N} cavities from rest")
    b = Batch(_problems(cases, n), device=dev)
    b.autotune(10)                  # the probe's result, from the cache: the timed batch runs it
    rec["tiling_timed"] = b.tiling()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _init_cold(b, N, n, dev)
    rc = batch_run_to_steady(b, tol=a.tol, max_steps=a.cap, check_every=100, log=_progress("cold"))
    torch.cuda.synchronize()
    rec["cold_batch"] = {"seconds": time.perf_counter() - t0, "steps": rc["steps_to_converge"].tolist(),
                         "status": rc["status"].tolist(), "res_u": rc["stats"]["res_u"].tolist(),
                         "res_phi": rc["stats"]["res_phi"].tolist()}
    del b
    rec["single_seconds_per_step"] = single_step_seconds(cases[0], n)
    say(f"cold batch {rec['cold_batch']['seconds']:.1f} s, converged "
        f"{sum(x == 'converged' for x in rc['status'])}/{N}; single lattice "
        f"{1e6 * rec['single_seconds_per_step']:.1f} us/step")
    _dump(rec, a.out)


def _omega_reference_from(states, cases, idx, n, tol, cap, dev):
    """FP64 steady states of the chosen cases, continued from the given FP64 populations
    (a converged FP32 state) by the parity-pinned FP64 path until r < tol or cap steps.
    A steady cavity flow at these Reynolds numbers is one fixed point, so the FP64 run
    ends at the FP64 steady state; starting near it makes it cheap for every Re."""
    out = []
    for j, i in enumerate(idx):
        lat = Lattice(W.cavity_problem(n, *cases[i], storage="f64"), device=dev)
        f, g = states[j]
        lat.set_populations(f, g, step=0)
        r = run_to_steady(lat, tol=tol, max_steps=cap, check_every=100)
        e = lat.extract(["wz", "phi"])
        out.append((e["wz"].cpu().numpy(), e["phi"].cpu().numpy(), r["status"], r["steps"]))
        del lat
    return out


def _spread(cases, k):
    """k case indices spread evenly over the Reynolds-number range (sorted by Re)."""
    order = np.argsort([c[0] for c in cases])
    return [int(order[int(round(q))]) for q in np.linspace(0, len(cases) - 1, k)]


def _omega_reference(cases, idx, n, tol, cap, dev):
    """FP64 cold-start steady states of the chosen cases (the parity-pinned FP64 path)."""
    b = Batch(_problems([cases[i] for i in idx], n, storage="f64"), device=dev)
    _init_cold(b, len(idx), n, dev)
    r = batch_run_to_steady(b, tol=tol, max_steps=cap, check_every=100, log=_progress("f64"))
    out = []
    for j in range(len(idx)):
        e = b.extract(j, ["wz", "phi"])
        out.append((e["wz"].cpu().numpy(), e["phi"].cpu().numpy(), r["status"][j]))
    return out


def cmd_warm(a):
    """Warm arm: prediction, fallback check, batch run; then omega of the warm-started
    steady states against FP64 cold-started ones for the a.n_omega lowest-Re cases."""
    dev = "cuda"
    n = a.n
    cases = W.surrogate_cases(a.n_eval, W.SURROGATE_HELDOUT_SEED0)
    N = len(cases)
    re = torch.tensor([c[0] for c in cases], dtype=torch.float32, device=dev)
    u = torch.tensor([c[1] for c in cases], dtype=torch.float32, device=dev)
    rec = {"arm": "warm", "n_eval": N, "side": n, "cap": a.cap, "tol": a.tol, "cases": cases}
    if a.weights:
        net, meta = S.load_weights(a.weights, device=dev)
        rec["weights"] = {k: (v.item() if v.ndim == 0 else v.tolist()) for k, v in meta.items()}
    else:
        net = S.UNet(base=32, levels=4, device=dev, seed=a.seed)
        rec["weights"] = "untrained"
    if a.corrupt:
        net.w.mul_(a.corrupt)     # forced-fallback rehearsal: scaled weights
        net.cast()
        rec["corrupt"] = a.corrupt
    probe = Batch(_problems(cases, n), device=dev)
    rec["tiling"] = probe.autotune(10)
    del probe
    say(f"warm batch ({rec['weights'] if isinstance(rec['weights'], str) else 'trained'} network)")
    b = Batch(_problems(cases, n), device=dev)
    b.autotune(10)                  # the probe's result, from the cache: the timed batch runs it
    rec["tiling_timed"] = b.tiling()
    # one untimed prediction compiles nothing but touches every buffer once
    S.predict_batch_fields(net, re[:16], u[:16], n, n)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fb = S.warm_start_batch(net, b, re, u, _cold(n), check_steps=100, fallback_tol=1e-2)
    torch.cuda.synchronize()
    t_ws = time.perf_counter() - t0
    rw = batch_run_to_steady(b, tol=a.tol, max_steps=a.cap - 100, check_every=100, log=_progress("warm"))
    torch.cuda.synchronize()
    steps_w = np.where(rw["steps_to_converge"] >= 0, rw["steps_to_converge"] + 100, -1)
    rec["warm_batch"] = {"seconds": time.perf_counter() - t0, "seconds_warm_start": t_ws, "fallbacks": int(fb.sum()),
                         "fallback_mask": fb.tolist(), "steps": steps_w.tolist(), "status": rw["status"].tolist(),
                         "res_u": rw["stats"]["res_u"].tolist(), "res_phi": rw["stats"]["res_phi"].tolist()}
    say(f"warm batch {rec['warm_batch']['seconds']:.1f} s (warm start {t_ws:.2f} s), fallbacks {int(fb.sum())}, "
        f"converged {sum(x == 'converged' for x in rw['status'])}/{N}")
    if a.n_omega > 0:
        conv_idx = [i for i in range(N) if rw["status"][i] == "converged"]
        idx = [conv_idx[j] for j in _spread([cases[i] for i in conv_idx], a.n_omega)]
        warm_w = {i: b.extract(i, ["wz"])["wz"].cpu().numpy() for i in idx}
        states = [b.get_populations(i) for i in idx]
        del b
        ref = _omega_reference_from(states, cases, idx, n, a.omega_tol, a.omega_cap, dev)
        errs = []
        for i, (w64, phi64, st, steps) in zip(idx, ref):
            m = phi64 >= 0.1
            e = float(np.linalg.norm((warm_w[i] - w64)[m]) / np.linalg.norm(w64[m]))
            errs.append({"case": i, "re": cases[i][0], "err": e, "f64_status": str(st), "f64_steps": int(steps),
                         "warm_status": rec["warm_batch"]["status"][i]})
        rec["omega_vs_f64"] = errs
        rec["omega_reference"] = (f"FP64 path continued from the warm FP32 steady state to r < {a.omega_tol:g} "
                                  f"(cap {a.omega_cap} steps); {a.n_omega} converged cases spread over Re")
        say("omega vs FP64:", [(round(x["re"]), round(x["err"], 6), x["f64_status"]) for x in errs])
    _dump(rec, a.out)


def _dump(rec, path):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)


def report(cold, warm):
    """Summary of the study from the two arm records (dicts)."""
    cap = cold["cap"]
    sc = np.asarray(cold["cold_batch"]["steps"])
    sw = np.asarray(warm["warm_batch"]["steps"])
    cc = np.asarray(cold["cold_batch"]["status"]) == "converged"
    cw = np.asarray(warm["warm_batch"]["status"]) == "converged"
    both = cc & cw
    single = cold["single_seconds_per_step"] * float(np.where(cc, sc, cap).sum())
    out = {
        "n_eval": cold["n_eval"], "cap": cap, "tol": cold["tol"],
        "converged_cold": int(cc.sum()), "converged_warm": int(cw.sum()), "converged_both": int(both.sum()),
        "fallbacks": warm["warm_batch"]["fallbacks"],
        "seconds_cold_single": single,
        "seconds_cold_batch": cold["cold_batch"]["seconds"],
        "seconds_warm_batch": warm["warm_batch"]["seconds"],
        "speedup_warm_batch_vs_cold_single": single / warm["warm_batch"]["seconds"],
        "speedup_warm_batch_vs_cold_batch": cold["cold_batch"]["seconds"] / warm["warm_batch"]["seconds"],
        "speedup_cold_batch_vs_cold_single": single / cold["cold_batch"]["seconds"],
    }
    if both.any():
        out["median_steps_cold_over_warm"] = float(np.median(sc[both] / sw[both]))
        out["total_steps_cold_over_warm_both"] = float(sc[both].sum() / sw[both].sum())
    if "omega_vs_f64" in warm:
        out["omega_vs_f64_max"] = max(x["err"] for x in warm["omega_vs_f64"])
    return out


def cmd_report(a):
    with open(a.cold) as f:
        cold = json.load(f)
    with open(a.warm) as f:
        warm = json.load(f)
    print(json.dumps(report(cold, warm), indent=1))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--n-train", type=int, default=512)
    t.add_argument("--n", type=int, default=N_SIDE)
    t.add_argument("--cap", type=int, default=400_000)
    t.add_argument("--iters", type=int, default=4000)
    t.add_argument("--batch", type=int, default=8)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--data-seconds", type=float, default=None, help="wall-time bound of the data generation")
    t.add_argument("--warm-data", default=None,
                   help="weights of a network that warm-starts the data generation (targets stay solver steady states)")
    t.add_argument("--seed", type=int, default=0)
    t.add_argument("--out", required=True)
    for name in ("cold", "warm"):
        e = sub.add_parser(name)
        e.add_argument("--n-eval", type=int, default=200)
        e.add_argument("--n", type=int, default=N_SIDE)
        e.add_argument("--cap", type=int, default=1_000_000)
        e.add_argument("--tol", type=float, default=1e-8)
        e.add_argument("--out", required=True)
        if name == "warm":
            e.add_argument("--weights", default=None)
            e.add_argument("--seed", type=int, default=0)
            e.add_argument("--n-omega", type=int, default=8)
            e.add_argument("--omega-tol", type=float, default=1e-10)
            e.add_argument("--omega-cap", type=int, default=400_000)
            e.add_argument("--corrupt", type=float, default=0.0)
    r = sub.add_parser("report")
    r.add_argument("cold")
    r.add_argument("warm")
    a = ap.parse_args(argv)
    if a.cmd == "report":
        return cmd_report(a)
    if not torch.cuda.is_available():
        sys.exit("the surrogate study needs a GPU")
    {"train": cmd_train, "cold": cmd_cold, "warm": cmd_warm}[a.cmd](a)


if __name__ == "__main__":
    main()
