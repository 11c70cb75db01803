"""Per-parity step times of one lattice over its launch settings.

    python3 -m paper_1908_06742_amd.launch_sweep --storage f32,f64 --size 8192 \
        [--kind periodic|cavity] [--tiles 128] [--widths 32,64] [--caps all | 2/2,1/1]

For every storage, tile width, lane-offset width and pair of resident-workgroup caps
(even / odd step; 0 = no cap) it prints the mean time of the even and of the odd step
kernel, from HIP events around single eager launches on the lattice's stream, and the
fastest setting per parity.  Results do not depend on these settings (tested), so the
sweep can run on any state: the decaying vortex field (periodic) or a cavity at rest
with a moving lid.
"""
from __future__ import annotations

import argparse
import itertools

import numpy as np
import torch

import workloads as W

from .lattice import Lattice

BYTES_PER_NODE = {"f64": 288, "f32": 144, "f16": 72, "bf16": 72, "bf16sr": 72}


def per_parity(lat, pairs=6):
    """Mean ms of the even and of the odd step kernel over `pairs` launches each."""
    st = torch.cuda.current_stream() if lat.stream is None else lat.stream
    if lat.step_count % 2:
        lat.step(1)
    lat.step(2)
    ev = {0: [], 1: []}
    for _ in range(2 * pairs):
        par = lat.step_count % 2
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        lat.step(1)
        b.record(st)
        ev[par].append((a, b))
    torch.cuda.synchronize()
    return [sum(x.elapsed_time(y) for x, y in ev[p]) / len(ev[p]) for p in (0, 1)]


def _caps(spec):
    if spec == "all":
        return list(itertools.product((0, 1, 2, 3), repeat=2))
    return [tuple(int(c) for c in pair.split("/")) for pair in spec.split(",")]


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--size", type=int, default=8192)
    ap.add_argument("--kind", choices=("periodic", "cavity"), default="periodic")
    ap.add_argument("--tiles", default="", help="tile widths (default: the library's choice)")
    ap.add_argument("--widths", default="32,64", help="lane-offset widths")
    ap.add_argument("--caps", default="all", help="'all' or pairs such as 2/2,1/1")
    ap.add_argument("--pairs", type=int, default=6, help="launches per parity and setting")
    args = ap.parse_args(argv)
    n = args.size
    if args.kind == "periodic":
        fields = W.VortexField(L=n).eval_grid(np.arange(n), np.arange(n), device="cuda")
    for storage in args.storage.split(","):
        if args.kind == "periodic":
            pr, fl = W.vortex_problem(n, storage=storage), fields
        else:
            pr, fl = W.cavity_problem(n, 20000.0, 0.1, storage=storage), W.cavity_fields(n, 0.5)
        lat = Lattice(pr, device="cuda").init(*fl)
        if storage != "bf16sr":
            lat.set_graph(0)
        bpn = BYTES_PER_NODE[storage]
        tiles = [int(t) for t in args.tiles.split(",")] if args.tiles else [lat.tile_width]
        best = {0: (float("inf"), None), 1: (float("inf"), None)}
        print(f"{args.kind} {storage} {n}^2, {lat.layout} rows", flush=True)
        for tw in tiles:
            lat.set_tile_width(tw)
            for aw in (int(w) for w in args.widths.split(",")):
                try:
                    lat.set_address_width(aw)
                except RuntimeError as e:   # 32-bit offsets need planes below 4 GiB
                    print(f"  offsets {aw}: {e}", flush=True)
                    continue
                for e, o in _caps(args.caps):
                    lat.set_workgroups_per_cu(e, o)
                    te, to = per_parity(lat, args.pairs)
                    for par, t, cap in ((0, te, e), (1, to, o)):
                        if t < best[par][0]:
                            best[par] = (t, (tw, aw, cap))
                    gbs = bpn * n * n / ((te + to) / 2 * 1e-3) / 1e9
                    print(f"  tile {tw} offsets {aw} caps {e}/{o}: even {te:.4f} odd {to:.4f} mean {(te + to) / 2:.4f} ms "
                          f"({gbs:.0f} GB/s)", flush=True)
        (te, se), (to, so) = best[0], best[1]
        print(f"  best even {te:.4f} ms (tile, offsets, cap) {se}; best odd {to:.4f} ms {so}", flush=True)
        del lat
        torch.cuda.empty_cache()


if __name__ == "__main__":
    main()
