"""Throughput of the fused two-lattice DDF step on one MI355X.

Workload: the periodic 8192 x 8192 decaying vortex field (seeded random Fourier
velocity modes 4 <= |k| <= 16 with max |u| = 0.02, 1024 Gaussian scalar blobs with
sigma = 32 cells), FP32 offset population storage, FP32 compute, tau = 0.8,
tau_phi = 0.7, beta = (1, 0.9).  One benchmark step is one pass of the hot path:
100 fused stream-and-collide time steps of both lattices, one FP64 reduction
(mass, scalar, residual, non-finite count) and one extraction of rho, u, phi, S and
omega.  `value` is MLUPS: fluid+scalar node-updates per second / 1e6, inputs
resident in HBM.  The roofline object reports the step kernel's algorithmic HBM
bandwidth (144 B per node-update in FP32: 18 populations read and written) from
HIP events around its launches, against the 8 TB/s HBM3E peak.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
LB_STEPS_PER_STEP = 100
BYTES_PER_NODE = {"f64": 288, "f32": 144, "f16": 72, "bf16": 72, "bf16sr": 72}
COUNTERS_FILE = os.path.join(ROOT, "profiles", "step_vortex8192_f32_counters.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1908_06742_amd", "csrc", n)
                  for n in ("ddf.hip", "ddf_kernels.hpp", "ddf_device.hpp", "ddf_handle.hpp", "ddf_step_launch.hpp",
                            "ddf_step_row.hip", "ddf_step_il.hip")]


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(nodes, tile_width):
    """HBM bytes per step launch from the committed rocprofv3 counter summary, or None
    when the kernel sources or the tile width changed since the counters were taken."""
    try:
        d = json.load(open(COUNTERS_FILE))
    except (OSError, ValueError):
        return None
    if d.get("kernel_hash") != kernel_hash() or d.get("nodes") != nodes or d.get("tile_width") != tile_width:
        return None
    return d.get("bytes_per_launch")


def time_parities(lat, stream, pairs=20):
    """Mean duration of one even and one odd step launch (HIP events around each eager
    launch on the lattice's stream), then the graph replays are restored."""
    import torch

    graphs = lat.problem.force_kind != "pulsatile" and lat.problem.storage != "bf16sr"
    if graphs:
        lat.set_graph(0)
    if lat.step_count % 2:
        lat.step(1)
    lat.step(2)
    torch.cuda.synchronize()
    ev = {0: [], 1: []}
    for _ in range(2 * pairs):
        par = lat.step_count % 2
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        lat.step(1)
        e1.record(stream)
        ev[par].append((e0, e1))
    torch.cuda.synchronize()
    if graphs:
        lat.set_graph(LB_STEPS_PER_STEP)
    return {p: sum(a.elapsed_time(b) for a, b in v) / len(v) for p, v in ev.items()}


def time_pattern(lat, stream, caps=(1, 2, 3), launches=8):
    """The step's access pattern without its collision (ddf_pattern_probe) on the
    lattice's own populations: mean ms per launch of each parity at each cap on resident
    workgroups per CU (an even number of launches per parity restores the populations)."""
    import torch

    out = {}
    for cap in caps:
        row = {}
        for par in (0, 1):
            lat.pattern_probe(par, cap)     # warm-up (and the pair to the odd count below)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(launches - 1):
                lat.pattern_probe(par, cap)
            e1.record(stream)
            e1.synchronize()
            row[par] = e0.elapsed_time(e1) / (launches - 1)
        out[cap] = row
    return out


def run_gpu(L, storage, steps, warmup, lb_steps=LB_STEPS_PER_STEP, tile_width=None, scalar_model="mrt",
            pulsatile=False, time_extract=False, parity_steps=False, pattern=None):
    import numpy as np
    import torch

    import workloads as W
    from paper_1908_06742_amd import Lattice

    vf = W.VortexField(L=L) if L == 8192 else W.VortexField(L=L, sigma=32.0 * L / 8192, n_blobs=max(16, 1024 * L * L // (8192 * 8192)))
    pr = W.vortex_problem(L, storage=storage, scalar_model=scalar_model)
    if pulsatile:
        # time-periodic uniform body force (the Womersley forcing), small against the field
        pr = pr.with_(force_kind="pulsatile", force=(1e-6, 0.0), force_omega=2.0 * np.pi / 1000.0)
    fields = vf.eval_grid(np.arange(L), np.arange(L), device="cuda")
    lat = Lattice(pr, device="cuda").init(*fields)
    if tile_width:
        lat.set_tile_width(tile_width)
    tile_width = lat.tile_width
    launch = {"layout": lat.layout, "address_width": lat.address_width,
              "workgroups_per_cu": list(lat.workgroups_per_cu)}
    del fields
    out = torch.empty((16, L, L), dtype=torch.float32, device="cuda")
    names = ["rho", "ux", "uy", "phi", "Sxx", "Syy", "Sxy", "wz"]
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()

    last = {}

    def one(kernel_events=None):
        if kernel_events is not None:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
        lat.step(lb_steps)
        if kernel_events is not None:
            e1.record(stream)
            kernel_events.append((e0, e1))
        last.update(lat.reduce())       # synchronises the stream
        lat.extract(names, out=out)

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    evs = []
    t0 = time.perf_counter()
    for _ in range(steps):
        one(evs)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kern_ms = sum(a.elapsed_time(b) for a, b in evs) / (steps * lb_steps)
    stats = dict(last)
    parity_ms = time_parities(lat, stream) if parity_steps else None
    pattern_ms = time_pattern(lat, stream) if (parity_steps if pattern is None else pattern) else None
    extract_ms = None
    if time_extract:
        # all 16 outputs (rho, u, phi, S, omega, gradients, Q, R, Lamb vector) in FP32
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(5):
            lat.extract(out=out)
        e1.record(stream)
        e1.synchronize()
        extract_ms = e0.elapsed_time(e1) / 5
    nodes = L * L
    return {
        "nodes": nodes,
        "seconds": dt,
        "mlups": nodes * lb_steps * steps / dt / 1e6,
        "ms_per_step": 1e3 * dt / steps,
        "kernel_ms": kern_ms,
        "stats": stats,
        "tile_width": tile_width,
        "launch": launch,
        "extract_ms": extract_ms,
        "parity_ms": parity_ms,
        "pattern_ms": pattern_ms,
    }


def run_cavity(n=1024, cap=200_000, tol=1e-8):
    """Lid-driven cavity n^2, Re = 1000, U = 0.1, FP32 offset storage, phi = 1 on the lid
    and 0 on the other walls, from rest until r < tol or `cap` steps (residual check
    every 100 steps).  Its 75 MB of populations stay in the 256 MB Infinity Cache, so
    this rate is not an HBM figure.  omega is compared with the centred-difference curl
    of the extracted velocity over interior nodes (two cells from the walls) with
    phi >= 0.1, and over the central quarter: the extraction carries
    the second-order scalar-curvature term the paper's relations drop, divided by phi,
    which the walls at phi = 0 make large."""
    import torch

    import workloads as W
    from paper_1908_06742_amd import Lattice
    from paper_1908_06742_amd.steady import run_to_steady

    pr = W.cavity_problem(n, 1000.0, 0.1, storage="f32")
    lat = Lattice(pr, device="cuda").init(*W.cavity_fields(n))
    m0 = lat.reduce()["mass"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = run_to_steady(lat, tol=tol, max_steps=cap, check_every=100)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    s = lat.reduce(raise_nonfinite=False)
    e = lat.extract(["ux", "uy", "phi", "wz"])
    ux, uy, phi, wz = e["ux"], e["uy"], e["phi"], e["wz"]
    curl = torch.zeros_like(wz)
    curl[1:-1, 1:-1] = 0.5 * (uy[1:-1, 2:] - uy[1:-1, :-2]) - 0.5 * (ux[2:, 1:-1] - ux[:-2, 1:-1])
    # the second-order scalar-curvature term the paper's n5 relation drops:
    # -2 c^2 [(1/w6 - 1/2) + (1/w7 - 1/2)] d_x d_y phi / ((beta1 - beta2) phi), with the
    # mixed derivative of the extracted phi by centred differences
    dxy = torch.zeros_like(phi)
    dxy[1:-1, 1:-1] = 0.25 * (phi[2:, 2:] - phi[2:, :-2] - phi[:-2, 2:] + phi[:-2, :-2])
    w6, w7 = pr.omega_phi_hi[3], pr.omega_phi_hi[4]
    pred = -2.0 * pr.cs2phi * ((1.0 / w6 - 0.5) + (1.0 / w7 - 0.5)) * dxy / ((pr.beta1 - pr.beta2) * phi)

    def err(mask, w=wz):
        return float(torch.linalg.norm((w - curl)[mask]) / torch.linalg.norm(curl[mask]))

    m = torch.zeros_like(phi, dtype=torch.bool)
    m[2:-2, 2:-2] = True
    m &= phi >= 0.1
    c = torch.zeros_like(m)
    c[n // 4:3 * n // 4, n // 4:3 * n // 4] = True
    c &= phi >= 0.1
    ew, ec = err(m), (err(c) if bool(c.any()) else None)
    ewc = err(m, wz - pred)
    ecc = err(c, wz - pred) if bool(c.any()) else None
    # the term alone, against the whole difference
    share = float(torch.linalg.norm(pred[m]) / torch.linalg.norm((wz - curl)[m]))
    # the step kernels alone (per parity), and the same accesses without the collision;
    # bytes per second of a cache-resident lattice, not an HBM figure
    stream = torch.cuda.current_stream()
    par = time_parities(lat, stream)
    pat = time_pattern(lat, stream)
    nb = BYTES_PER_NODE["f32"] * n * n
    pg = {cap: nb / (0.5 * (v[0] + v[1]) * 1e-3) / 1e9 for cap, v in pat.items()}
    pcap = max(pg, key=pg.get)
    kg = nb / (0.5 * (par[0] + par[1]) * 1e-3) / 1e9
    return {"workload": f"lid-driven cavity {n}^2, Re 1000, U 0.1, f32, to r < {tol:g} or {cap} steps",
            "mlups": round(n * n * r["steps"] / dt / 1e6, 1), "steps": r["steps"], "status": r["status"],
            "seconds": round(dt, 3), "res_u": r["res_u"], "res_phi": r["res_phi"],
            "mass_drift_rel": abs(s["mass"] - m0) / m0, "nonfinite": s["nonfinite"],
            "omega_vs_fd_curl_rel_l2": ew, "omega_vs_fd_curl_rel_l2_centre_quarter": ec,
            "omega_minus_curvature_term_vs_fd_curl_rel_l2": ewc,
            "omega_minus_curvature_term_vs_fd_curl_rel_l2_centre_quarter": ecc,
            "curvature_term_over_difference_l2": share,
            "kernel_ms_even": round(par[0], 4), "kernel_ms_odd": round(par[1], 4), "kernel_gbs": round(kg, 1),
            "pattern_gbs": round(pg[pcap], 1), "pattern_wg_per_cu": pcap, "frac_of_pattern": round(kg / pg[pcap], 4)}


def stream_ceilings(nbytes=2 << 30, reps=5):
    """What plain streams reach on this device, from the library's reference kernels
    (ddf_bandwidth_probe): the best copy (read + write bytes per second), read-only
    and write-only pass over `nbytes` (8x the 256 MB Infinity Cache) across their
    launch variants, plus torch's own device-to-device copy for comparison."""
    import ctypes as C

    import torch

    from paper_1908_06742_amd import _lib as L

    lib = L.lib()
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    sp = C.c_void_p(stream.cuda_stream)

    def best_ms(fn):
        fn()
        best = 1e30
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1))
        return best

    out = {"bytes": nbytes}
    for kind, name, factor in ((L.PROBE_COPY, "copy", 2.0), (L.PROBE_READ, "read", 1.0), (L.PROBE_WRITE, "write", 1.0)):
        rows = []
        for unroll in (1, 2, 4, 8):
            for nt in (0, 1):
                def fn():
                    L.check(lib.ddf_bandwidth_probe(kind, unroll, nt, C.c_void_p(src.data_ptr()),
                                                    C.c_void_p(dst.data_ptr()), nbytes, sp))
                ms = best_ms(fn)
                rows.append((factor * nbytes / (ms * 1e-3) / 1e9, unroll, nt))
        gbs, unroll, nt = max(rows)
        out[f"{name}_gbs"] = round(gbs, 1)
        out[f"{name}_variant"] = {"unroll": unroll, "nontemporal": nt}
    out["torch_copy_gbs"] = round(2.0 * nbytes / (best_ms(lambda: dst.copy_(src)) * 1e-3) / 1e9, 1)
    del src, dst
    return out


def run_batch(steps=20000, count=256):
    """256 cavities and channels of sides 64..512, Re 100..5000, U 0.05..0.1 (seeded),
    FP32 in packed rows, autotuned tiling and cache policy, graph-captured runs of 100
    steps."""
    import numpy as np
    import torch

    import workloads as W
    from paper_1908_06742_amd import Batch

    inst = W.batch_instances(count)
    b = Batch([i.problem for i in inst], device="cuda")
    tune = b.autotune(steps_per_trial=10)
    fields = [W.rest_fields(i.nx, i.ny, 1.0, 0.0 if i.kind == "cavity" else 0.5) for i in inst]
    b.init(fields)
    b.step(200)
    b.reduce()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = b.step_reduce(steps)
    dt = time.perf_counter() - t0
    nodes = b.total_nodes
    # the step kernel per parity (eager launches) and the same accesses without the
    # collision (ddf_batch_pattern_probe; 8 launches per parity restore the populations)
    stream = torch.cuda.current_stream()
    b.set_graph(0)
    if b.step_count % 2:
        b.step(1)

    def mean_ms(fn, n):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(n):
            fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / n

    pair = mean_ms(lambda: b.step(2), 10)
    pat = [0.0, 0.0]
    for par in (0, 1):
        b.pattern_probe(par)
        pat[par] = mean_ms(lambda: b.pattern_probe(par), 7)
    b.set_graph(100)
    kg = 144.0 * nodes / (0.5 * pair * 1e-3) / 1e9
    pg = 144.0 * nodes / (0.5 * (pat[0] + pat[1]) * 1e-3) / 1e9
    return {"instances": count, "nodes": nodes, "mlups": round(nodes * steps / dt / 1e6, 1), "steps": steps,
            "seconds": round(dt, 3), "tiling": b.tiling(), "nontemporal": list(b.nontemporal),
            "autotune_ms_per_step": tune["ms_per_step"],
            "nonfinite_instances": int(np.sum(s["nonfinite"] > 0)),
            "hbm_gbs": round(144.0 * nodes * steps / dt / 1e9, 1),
            "kernel_ms_per_step": round(0.5 * pair, 4), "kernel_gbs": round(kg, 1),
            "pattern_ms": [round(pat[0], 4), round(pat[1], 4)], "pattern_gbs": round(pg, 1),
            "frac_of_pattern": round(kg / pg, 4)}


def run_surrogate(count=16, cap=400_000):
    """Time to r < 1e-8 of `count` held-out 256^2 cavities spread evenly over the Re
    range (seeds 100000..100199, every 200/count-th by Re), FP32: cold from rest one
    lattice at a time (each stepped alone on the GPU with the residual check every 100
    steps, as run), cold from rest in one batch, and warm from the shipped network's
    prediction in one batch (inference and the fallback check inside the timed region).
    Instances that reach the cap count with the cap."""
    import numpy as np
    import torch

    import workloads as W
    from paper_1908_06742_amd import Batch, Lattice
    from paper_1908_06742_amd import surrogate as S
    from paper_1908_06742_amd.steady import batch_run_to_steady, run_to_steady

    n = 256
    held = W.surrogate_cases(200, W.SURROGATE_HELDOUT_SEED0)
    order = sorted(range(len(held)), key=lambda i: held[i][0])
    cases = [held[order[int(round(q))]] for q in np.linspace(0, len(held) - 1, count)]
    probs = [W.cavity_problem(n, re, u) for re, u in cases]
    re = torch.tensor([c[0] for c in cases], dtype=torch.float32, device="cuda")
    u = torch.tensor([c[1] for c in cases], dtype=torch.float32, device="cuda")
    Batch(probs, device="cuda").autotune(10)
    net, _ = S.load_weights(os.path.join(ROOT, "paper_1908_06742_amd", "weights", "unet_cavity256.npz"))
    S.predict_batch_fields(net, re, u, n, n)       # first call allocates the activations
    # cold, one lattice at a time
    single_steps, single_conv = [], 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for pr in probs:
        lat = Lattice(pr, device="cuda").init(*W.cavity_fields(n))
        r1 = run_to_steady(lat, tol=1e-8, max_steps=cap, check_every=100)
        single_steps.append(r1["steps"])
        single_conv += r1["status"] == "converged"
        del lat
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t0
    # cold, one batch
    b = Batch(probs, device="cuda")
    b.autotune(10)                                  # cached: applies the probe's tiling
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    z = torch.zeros((count, n, n), dtype=torch.float64, device="cuda")
    b.init_device(torch.ones_like(z), z, z, z)
    rc = batch_run_to_steady(b, tol=1e-8, max_steps=cap, check_every=100)
    torch.cuda.synchronize()
    t_cold = time.perf_counter() - t0
    del b
    # warm, one batch
    b = Batch(probs, device="cuda")
    b.autotune(10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fb = S.warm_start_batch(net, b, re, u, lambda i: W.cavity_fields(n))
    rw = batch_run_to_steady(b, tol=1e-8, max_steps=cap - 100, check_every=100)
    torch.cuda.synchronize()
    t_warm = time.perf_counter() - t0
    sc = np.where(rc["steps_to_converge"] >= 0, rc["steps_to_converge"], cap)
    sw = np.where(rw["steps_to_converge"] >= 0, rw["steps_to_converge"] + 100, cap)
    return {"workload": f"{count} held-out 256^2 cavities spread over Re {cases[0][0]:.0f}..{cases[-1][0]:.0f}, "
                        f"FP32, to r < 1e-8 (cap {cap})",
            "re": [round(c[0], 1) for c in cases],
            "seconds_cold_single": round(t_single, 2), "seconds_cold_batch": round(t_cold, 2),
            "seconds_warm_batch": round(t_warm, 2), "speedup_vs_cold_single": round(t_single / t_warm, 2),
            "speedup_vs_cold_batch": round(t_cold / t_warm, 2), "fallbacks": int(fb.sum()),
            "converged_cold_single": int(single_conv),
            "converged_cold": int(np.sum(rc["status"] == "converged")),
            "converged_warm": int(np.sum(rw["status"] == "converged")),
            "steps_cold_over_warm": round(float(sc.sum() / sw.sum()), 2)}


BF16_PEAK_TFLOPS = 2500.0


def unet_flops_per_sample(H=256, W=256, base=32, levels=4):
    """Matrix-core FLOPs of one training sample (forward, data gradient, weight gradient)
    of the surrogate U-Net as the kernels execute it (channels padded to 32)."""
    from paper_1908_06742_amd.surrogate import layer_table, _pad

    fwd = dgrad = 0
    for name, ci, co, _ in layer_table(base, levels):
        lvl = 0 if name == "head" else int(name[3])
        cip = 32 if name == "enc0a" else _pad(ci)
        f = 2.0 * 9 * cip * _pad(co) * (H >> lvl) * (W >> lvl)
        fwd += f
        if name != "enc0a":
            dgrad += f
    return fwd, fwd + dgrad + fwd


def unet_bound_us(batch=8, H=256, W=256, base=32, levels=4):
    """Lower bound on one training iteration and on one forward pass of the surrogate
    U-Net (microseconds): every kernel at the larger of its matrix-core time at the dense
    BF16 peak and its HBM time at 8 TB/s for the bytes it must move (activations in and
    out once, as the kernels store them: channels padded to 32, BF16; weights, Adam
    state and the loss target once), summed over the kernels of an iteration."""
    from paper_1908_06742_amd.surrogate import layer_table, _pad

    pk, bw = BF16_PEAK_TFLOPS * 1e12, HBM_PEAK_GBS * 1e9
    t = lambda fl, by: 1e6 * max(fl / pk, by / bw)   # noqa: E731
    fwd = train = 0.0
    nparam = 0
    ch = [base * 2 ** k for k in range(levels)]
    for name, ci, co, _ in layer_table(base, levels):
        lvl = 0 if name == "head" else int(name[3])
        cip, cop = (32 if name == "enc0a" else _pad(ci)), _pad(co)
        px = batch * (H >> lvl) * (W >> lvl)
        fl = 2.0 * 9 * cip * cop * px
        nparam += 9 * cip * cop + cop
        f = t(fl, 2 * px * (cip + cop))
        fwd += f
        train += f + t(fl, 2 * px * (cip + cop))                 # weight gradient: input and dY
        if name != "enc0a":
            train += t(fl, 2 * px * (cop + 2 * cip))             # data gradient: dY, mask, dX
    for k in range(1, levels):                                   # pooling, upsampling, adjoints
        hi, lo, c = batch * (H >> (k - 1)) * (W >> (k - 1)), batch * (H >> k) * (W >> k), ch[k - 1]
        fwd += t(0, 2 * c * (hi + lo))
        train += t(0, 2 * c * (hi + lo)) + t(0, 2 * c * (3 * hi + lo))
        cu = ch[k]
        fwd += t(0, 2 * cu * (hi + lo))
        train += t(0, 2 * cu * (hi + lo)) * 2
    px0 = batch * H * W
    inputs = t(0, 2 * 32 * px0)
    loss = t(0, px0 * (2 * 32 + 16 + 2 * 32))                    # head, target; dY of the head
    adam = t(0, nparam * (4 * 4 + 3 * 4))                        # w, g, m, v in; w, m, v out
    cast = t(0, nparam * (4 + 2 * 2))
    return {"train_us": round(train + inputs + loss + adam + cast, 1), "forward_us": round(fwd + inputs, 1)}


def run_unet(batch=8, iters=50):
    """One Adam training iteration of the surrogate U-Net on batch x 256^2 (forward, loss,
    backward, Adam, BF16 weight casts), timed with HIP events; and the forward alone."""
    import torch

    from paper_1908_06742_amd.surrogate import UNet

    H = W = 256
    net = UNet(base=32, levels=4, device="cuda", seed=0)
    re = torch.linspace(100, 5000, batch, device="cuda")
    u = torch.full((batch,), 0.08, device="cuda")
    tgt = torch.randn(batch * H * W * 4, device="cuda") * 0.1
    for _ in range(3):
        net.train_step(re, u, tgt, H, W, 1e-5)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()

    def timed(fn, n):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(n):
            fn()
        e1.record(st)
        e1.synchronize()
        return e0.elapsed_time(e1) / n

    t_train = timed(lambda: net.train_step(re, u, tgt, H, W, 1e-5), iters)
    net.inputs(re, u, H, W)
    t_fwd = timed(lambda: net.forward(batch, H, W), iters)
    f_fwd, f_train = unet_flops_per_sample(H, W)
    bound = unet_bound_us(batch, H, W)
    tf_train = batch * f_train / (t_train * 1e-3) / 1e12
    tf_fwd = batch * f_fwd / (t_fwd * 1e-3) / 1e12
    return {"workload": f"surrogate U-Net (4 levels, base 32, BF16 MFMA), batch {batch} x 256^2",
            "ms_per_train_iter": round(t_train, 3), "train_tflops": round(tf_train, 1),
            "ms_per_forward": round(t_fwd, 3), "forward_tflops": round(tf_fwd, 1),
            "peak_tflops": BF16_PEAK_TFLOPS, "train_frac": round(tf_train / BF16_PEAK_TFLOPS, 4),
            "forward_frac": round(tf_fwd / BF16_PEAK_TFLOPS, 4),
            # the iteration against the sum of its kernels' matrix-core or HBM bounds
            "bound_ms_per_train_iter": round(bound["train_us"] / 1e3, 3),
            "frac_of_bound_train": round(bound["train_us"] / 1e3 / t_train, 4),
            "bound_ms_per_forward": round(bound["forward_us"] / 1e3, 3),
            "frac_of_bound_forward": round(bound["forward_us"] / 1e3 / t_fwd, 4)}


def cpu_baseline(budget_s=12.0):
    """The FP64 oracle timed on the host cores on a bounded sample of the same
    workload: a 256 x 256 window of the vortex field run as a periodic lattice, in
    chunks of 20 steps until the time budget is spent."""
    import numpy as np

    import oracle
    import workloads as W

    n = 256
    nthreads = os.cpu_count() or 1
    vf = W.VortexField(L=8192)
    pr = W.vortex_problem(n, storage="f64")
    o = oracle.Oracle(pr, nthreads=nthreads)
    f, g = o.init(*vf.fields(0, 0, n, n))
    steps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        o.step(f, g, 20, steps)
        steps += 20
    dt = time.perf_counter() - t0
    return {"value": n * n * steps / dt / 1e6, "unit": "MLUPS", "cores": nthreads, "kind": "oracle",
            "sample": f"FP64 oracle, {n}x{n} window of the 8192^2 vortex field run as a periodic lattice, {steps} steps, "
                      f"{dt:.1f} s on {nthreads} OpenMP threads"}


def oracle_timing():
    """The FP64 oracle's MLUPS on one thread and on all threads: the 64^2 Taylor-Green
    vortex (1000 steps, whole run), the 1024^2 cavity (100 steps) and a 1024^2 window of
    the 8192^2 vortex field run as a periodic lattice (100 steps; the full field's time
    is this per-node rate times 64, extrapolated)."""
    import oracle
    import workloads as W

    nall = os.cpu_count() or 1
    vf = W.VortexField(L=8192)
    cases = [
        ("taylor_green_64_f64_1000", W.taylor_green_problem(64), W.taylor_green_fields(64, 0.01), 1000),
        ("cavity_1024_100", W.cavity_problem(1024, 1000.0, 0.1, storage="f64"), W.cavity_fields(1024), 100),
        ("vortex_window_1024_100", W.vortex_problem(1024, storage="f64"), vf.fields(0, 0, 1024, 1024), 100),
    ]
    out = {}
    for name, pr, fields, steps in cases:
        row = {}
        for nt in (1, nall):
            o = oracle.Oracle(pr, nthreads=nt)
            f, g = o.init(*fields)
            t0 = time.perf_counter()
            o.step(f, g, steps, 0)
            dt = time.perf_counter() - t0
            row[f"mlups_{nt}_threads"] = round(pr.nx * pr.ny * steps / dt / 1e6, 2)
        out[name] = row
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--size", type=int, default=8192)
    ap.add_argument("--storage", default="f32", choices=["f64", "f32", "f16", "bf16", "bf16sr"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the 1024^2 cavity, 256-instance batch and surrogate time-to-steady lines")
    ap.add_argument("--batch-steps", type=int, default=20000)
    ap.add_argument("--no-oracle-timing", action="store_true",
                    help="skip timing the oracle single-threaded and on all threads on the small workloads")
    ap.add_argument("--variants", action="store_true", help="also time FP16/BF16/FP64 storage of the same field")
    ap.add_argument("--tile-width", type=int, default=None, help="tile width of the single-lattice kernels")
    ap.add_argument("--only-extra", choices=["cavity", "batch", "surrogate", "unet"],
                    help="run one extra line alone and print it (for profiling runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 5 times (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        # 1 GiB copies: the runtime's, then the library's non-temporal copy probe
        import ctypes as C

        import torch

        from paper_1908_06742_amd import _lib as L
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        sp = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        for _ in range(5):
            L.check(L.lib().ddf_bandwidth_probe(L.PROBE_COPY, 1, 1, C.c_void_p(src.data_ptr()),
                                                C.c_void_p(dst.data_ptr()), 1 << 30, sp))
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_per_dispatch": 1 << 30, "copy_bytes_written_per_dispatch": 1 << 30}))
        return
    if args.only_extra:
        fn = {"cavity": run_cavity, "batch": lambda: run_batch(args.batch_steps), "surrogate": run_surrogate,
              "unet": run_unet}[args.only_extra]
        print(json.dumps({args.only_extra: fn()}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    print(f"[bench] {args.size}^2 {args.storage}: warmup {args.warmup}, timed {args.steps} steps "
          f"x {LB_STEPS_PER_STEP} LB steps", file=sys.stderr, flush=True)
    r = run_gpu(args.size, args.storage, args.steps, args.warmup, tile_width=args.tile_width, parity_steps=True)
    nodes = r["nodes"]
    bpn = BYTES_PER_NODE[args.storage]
    achieved = bpn * nodes / (r["kernel_ms"] * 1e-3) / 1e9
    traffic = measured_traffic(nodes, r["tile_width"]) if args.storage == "f32" and args.size == 8192 else None
    ceil = stream_ceilings()
    cgbs = ceil["copy_gbs"]
    pat = {cap: {"even_ms": round(v[0], 4), "odd_ms": round(v[1], 4),
                 "gbs": round(bpn * nodes / (0.5 * (v[0] + v[1]) * 1e-3) / 1e9, 1)} for cap, v in r["pattern_ms"].items()}
    pcap = max(pat, key=lambda c: pat[c]["gbs"])
    line = {
        "metric": "MLUPS (fluid+scalar D2Q9 node-updates per second / 1e6)",
        "value": round(r["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.storage,
        "data": "synthetic",
        "config": {
            "workload": f"periodic {args.size}x{args.size} decaying vortex field, {args.storage} offset population "
                        f"storage, {'f64' if args.storage == 'f64' else 'f32'} compute; one step = "
                        f"{LB_STEPS_PER_STEP} fused two-lattice LB steps + FP64 reduction + extraction",
            "nx": args.size, "ny": args.size, "lb_steps_per_step": LB_STEPS_PER_STEP,
            "tau": 0.8, "tau_phi": 0.7, "beta": [1.0, 0.9],
        },
        "roofline": {
            "bound": "hbm",
            "kernel": f"k_step<{args.storage}, MRT, periodic>",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "algorithmic_bytes_per_launch": bpn * nodes,
            "kernel_ms_per_launch": round(r["kernel_ms"], 4),
            "kernel_ms_even": round(r["parity_ms"][0], 4),
            "kernel_ms_odd": round(r["parity_ms"][1], 4),
            "gbs_even": round(bpn * nodes / (r["parity_ms"][0] * 1e-3) / 1e9, 1),
            "gbs_odd": round(bpn * nodes / (r["parity_ms"][1] * 1e-3) / 1e9, 1),
            "tile_width": r["tile_width"],
            "launch": r["launch"],
            "copy_gbs": cgbs,
            "frac_of_copy": round(achieved / cgbs, 4),
            "stream_ceilings": ceil,
            # the same loads and stores without the collision (ddf_pattern_probe), best
            # cap on resident workgroups per CU
            "pattern_gbs": pat[pcap]["gbs"],
            "pattern_wg_per_cu": pcap,
            "frac_of_pattern": round(achieved / pat[pcap]["gbs"], 4),
            "pattern_by_wg_per_cu": pat,
        },
        "final_stats": {k: r["stats"][k] for k in ("mass", "scalar", "res_u", "nonfinite")},
    }
    if not args.no_extras:
        print("[bench] extra: cavity 1024^2 f32", file=sys.stderr, flush=True)
        line["extras"] = {"cavity1024_f32": run_cavity()}
        print("[bench] extra: batch of 256 instances f32", file=sys.stderr, flush=True)
        line["extras"]["batch256_f32"] = run_batch(args.batch_steps)
        print("[bench] extra: surrogate warm start vs cold start", file=sys.stderr, flush=True)
        line["extras"]["surrogate256_time_to_steady"] = run_surrogate()
        print("[bench] extra: surrogate U-Net training step", file=sys.stderr, flush=True)
        line["extras"]["unet256_train_b8"] = run_unet()
    if args.variants:
        var = []
        cases = [dict(storage="f16"), dict(storage="bf16"), dict(storage="bf16sr"), dict(storage="f64"),
                 dict(storage="f32", scalar_model="srt"), dict(storage="f32", scalar_model="central"),
                 dict(storage="f32", scalar_model="cascaded"), dict(storage="f32", pulsatile=True),
                 dict(storage="f32", time_extract=True)]
        for c in cases:
            st = c["storage"]
            print(f"[bench] variant 8192^2 {c}", file=sys.stderr, flush=True)
            plain = len(c) == 1      # a storage format alone: also its access pattern without the collision
            v = run_gpu(8192, st, 3, 1, scalar_model=c.get("scalar_model", "mrt"), pulsatile=c.get("pulsatile", False),
                        time_extract=c.get("time_extract", False), pattern=plain)
            ach = BYTES_PER_NODE[st] * v["nodes"] / (v["kernel_ms"] * 1e-3) / 1e9
            row = {**c, "size": 8192, "mlups": round(v["mlups"], 1), "kernel_gbs": round(ach, 1),
                   "frac": round(ach / HBM_PEAK_GBS, 4), "tile_width": v["tile_width"], "launch": v["launch"]}
            if v["pattern_ms"]:
                pg = {cap: BYTES_PER_NODE[st] * v["nodes"] / (0.5 * (e + o) * 1e-3) / 1e9
                      for cap, (e, o) in ((k, (t[0], t[1])) for k, t in v["pattern_ms"].items())}
                best = max(pg, key=pg.get)
                row.update({"pattern_gbs": round(pg[best], 1), "pattern_wg_per_cu": best,
                            "frac_of_pattern": round(ach / pg[best], 4)})
            if v["extract_ms"] is not None:
                # reads both lattices once (half the step's bytes: 72 B/node in FP32) and
                # writes 16 FP32 outputs (64 B/node)
                eb = (BYTES_PER_NODE[st] // 2 + 64) * v["nodes"] / (v["extract_ms"] * 1e-3) / 1e9
                row.update({"extract_all_ms": round(v["extract_ms"], 3), "extract_gbs": round(eb, 1),
                            "extract_frac": round(eb / HBM_PEAK_GBS, 4)})
            var.append(row)
        line["variants"] = var
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline()
        if not args.no_oracle_timing:
            print("[bench] oracle timing (single thread and all threads)", file=sys.stderr, flush=True)
            line["cpu_baseline"]["oracle_timing"] = oracle_timing()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
