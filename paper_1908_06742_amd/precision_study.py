"""Error of reduced-precision population storage on the periodic decaying vortex field.

    python -m paper_1908_06742_amd.precision_study --n 8192 --steps 5000 --out precision.json

Every storage format runs the same seeded field (random Fourier streamfunction modes
4 <= |k| <= 16 scaled to max |u| = 0.02, scalar 1 + Gaussian blobs of sigma 32) for the
same number of steps; u, phi and omega_z are compared with the FP64-storage run, whose
arithmetic matches the FP64 oracle to 1e-12 per trajectory.  Errors are normwise
relative L2 over the whole lattice: |u - u64| / |u64| for the velocity vector,
|phi - phi64| / |phi64 - mean(phi64)| for the scalar (its variation, not its background)
and |w - w64| / |w64| for the vorticity over nodes with phi >= 0.1 (all of them here).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import torch

import workloads as W

from .lattice import Lattice


def say(*a):
    print(*a, flush=True)


def run(storage, n, steps, fields):
    pr = W.vortex_problem(n, storage=storage)
    lat = Lattice(pr, device="cuda").init(*fields)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = lat.extract(["ux", "uy", "phi", "wz"])
    res = {k: v.clone() for k, v in out.items()}
    stats = lat.reduce(raise_nonfinite=False)
    del lat, out
    torch.cuda.empty_cache()
    return res, dt, stats


def errors(a, ref):
    du = torch.sqrt(torch.sum((a["ux"] - ref["ux"]) ** 2 + (a["uy"] - ref["uy"]) ** 2))
    nu = torch.sqrt(torch.sum(ref["ux"] ** 2 + ref["uy"] ** 2))
    pv = ref["phi"] - ref["phi"].mean()
    m = ref["phi"] >= 0.1
    return {
        "u": float(du / nu),
        "phi": float(torch.linalg.norm(a["phi"] - ref["phi"]) / torch.linalg.norm(pv)),
        "omega": float(torch.linalg.norm((a["wz"] - ref["wz"])[m]) / torch.linalg.norm(ref["wz"][m])),
        "u_max_abs": float(torch.max(torch.abs(a["ux"] - ref["ux"])).item()),
        "omega_max_rel": float(torch.max(torch.abs(a["wz"] - ref["wz"])).item() / torch.max(torch.abs(ref["wz"])).item()),
    }


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--storages", default="f32,f16,bf16,bf16sr")
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    if not torch.cuda.is_available():
        sys.exit("the precision study needs a GPU")
    vf = W.VortexField(L=a.n)
    fields = vf.eval_grid(torch.arange(a.n).numpy(), torch.arange(a.n).numpy(), device="cuda")
    say(f"FP64 reference: {a.n}^2, {a.steps} steps")
    ref, dt64, st64 = run("f64", a.n, a.steps, fields)
    rec = {"n": a.n, "steps": a.steps, "seconds": {"f64": dt64}, "mass": {"f64": st64["mass"]}, "errors": {}}
    for s in a.storages.split(","):
        say(f"storage {s}")
        res, dt, st = run(s, a.n, a.steps, fields)
        rec["seconds"][s] = dt
        rec["mass"][s] = st["mass"]
        rec["errors"][s] = errors(res, ref)
        say(f"  {dt:.1f} s  " + "  ".join(f"{k} {v:.3e}" for k, v in rec["errors"][s].items()))
        del res
        torch.cuda.empty_cache()
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    with open(a.out, "w") as f:
        json.dump(rec, f, indent=1)


if __name__ == "__main__":
    main()
