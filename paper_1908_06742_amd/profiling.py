"""Summaries of rocprofv3 result databases (rocpd SQLite) for the step kernels.

Usage (each database from its own rocprofv3 run; see profiles/*.md for the commands):
  python -m paper_1908_06742_amd.profiling trace <run_results.db>
  python -m paper_1908_06742_amd.profiling sequence <run_results.db> --marker k_adam
  python -m paper_1908_06742_amd.profiling counters <fetch.db> <write.db> <copy_fetch.db> <copy_write.db> \
      --kernel k_step --nodes N --bytes-per-node B --tile-width T --out profiles/<name>_counters.json

FETCH_SIZE and WRITE_SIZE are reported by rocprofv3 in KiB per dispatch.  Each is
scaled by the ratio of the true byte count of a plain 1 GiB device copy to what the
same counter reads for that copy.
"""
from __future__ import annotations

import argparse
import json
import sqlite3
import sys


def kernel_stats(db):
    """Per-kernel dispatch count and durations (ns) from the kernel dispatch records."""
    con = sqlite3.connect(db)
    rows = con.execute("select name, count(*), sum(end - start), avg(end - start), min(end - start), "
                       "max(end - start) from kernels group by name order by sum(end - start) desc").fetchall()
    total = sum(r[2] for r in rows)
    return [dict(name=r[0], calls=r[1], total_ns=r[2], avg_ns=r[3], min_ns=r[4], max_ns=r[5],
                 percent=100.0 * r[2] / total) for r in rows]


def counter_means(db, counter):
    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, avg(value), count(*) from counters_collection where counter_name = ? "
                       "group by kernel_name", (counter,)).fetchall()
    return {r[0]: (r[1], r[2]) for r in rows}


def readable(name):
    """A mangled nested name the profiler left as is (_ZN<len><id>...E<params>) as
    scope::name(...); anything else unchanged."""
    if not name.startswith("_ZN"):
        return name
    parts, i = [], 3
    while i < len(name) and name[i].isdigit():
        j = i
        while j < len(name) and name[j].isdigit():
            j += 1
        k = int(name[i:j])
        ident = name[j:j + k]
        parts.append("(anonymous namespace)" if ident.startswith("_GLOBAL__N") else ident)
        i = j + k
    return "::".join(parts) + "(...)" if parts else name


def short(name, n=90):
    name = readable(name)
    return name if len(name) <= n else name[: n - 3] + "..."


def cmd_trace(args):
    st = kernel_stats(args.db)
    print(f"{'avg us':>10} {'min us':>10} {'max us':>10} {'calls':>6} {'%':>6}  kernel")
    for k in st[: args.top]:
        print(f"{k['avg_ns'] / 1e3:10.1f} {k['min_ns'] / 1e3:10.1f} {k['max_ns'] / 1e3:10.1f} {k['calls']:6d} "
              f"{k['percent']:6.2f}  {short(k['name'])}")


def cmd_counters(args):
    fetch = counter_means(args.fetch, "FETCH_SIZE")
    write = counter_means(args.write, "WRITE_SIZE")
    cf = counter_means(args.copy_fetch, "FETCH_SIZE")
    cw = counter_means(args.copy_write, "WRITE_SIZE")
    copy_name = [k for k in cf if args.copy_kernel in k][0]
    copy_kib = 1 << 20   # 1 GiB read and written per copy dispatch
    f_scale = copy_kib / cf[copy_name][0]
    w_scale = copy_kib / cw[copy_name][0]
    sel = [k for k in fetch if args.kernel in k]
    rows = []
    for k in sorted(sel):
        fb = fetch[k][0] * f_scale * 1024.0
        wb = write.get(k, (float("nan"), 0))[0] * w_scale * 1024.0
        rows.append(dict(kernel=k, dispatches=fetch[k][1], fetch_bytes=fb, write_bytes=wb))
    algo = args.nodes * args.bytes_per_node
    print(f"copy calibration: FETCH_SIZE x {f_scale:.4f}, WRITE_SIZE x {w_scale:.4f} (1 GiB copy, {copy_name})")
    print(f"algorithmic bytes per launch: {algo:.6e} ({args.bytes_per_node} B/node x {args.nodes} nodes)")
    for r in rows:
        tot = r["fetch_bytes"] + r["write_bytes"]
        print(f"{short(r['kernel'], 70)}: fetch {r['fetch_bytes']:.6e} B, write {r['write_bytes']:.6e} B, "
              f"total {tot:.6e} B = {tot / algo:.4f} x algorithmic ({r['dispatches']} dispatches)")
    mean_total = sum(r["fetch_bytes"] + r["write_bytes"] for r in rows) / len(rows)
    if args.out:
        import os
        sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
        import bench
        json.dump({"kernel_hash": bench.kernel_hash(), "nodes": args.nodes, "tile_width": args.tile_width,
                   "calibration_kernel": copy_name,
                   "bytes_per_launch": mean_total,
                   "algorithmic_bytes_per_launch": algo, "fetch_scale": f_scale, "write_scale": w_scale,
                   "per_parity": rows}, open(args.out, "w"), indent=1)
        print(f"wrote {args.out}")


def cmd_sequence(args):
    """The dispatches between the last two complete launches of a marker kernel (one
    training iteration between two optimizer steps, say): duration of each, their sum,
    the time the GPU runs at least one of them (kernels on several streams overlap) and
    the span from the end of the first marker to the end of the second."""
    con = sqlite3.connect(args.db)
    rows = con.execute("select name, start, end from kernels order by start").fetchall()
    marks = [i for i, r in enumerate(rows) if args.marker in r[0]]
    if len(marks) < 3:
        sys.exit(f"fewer than three launches of {args.marker!r}")
    i0, i1 = marks[-3], marks[-2]   # the last marker may close a shorter, different phase
    total = busy = 0.0
    reach = rows[i0][2]             # union of the intervals, swept in start order
    for name, start, end in rows[i0 + 1:i1 + 1]:
        total += (end - start) / 1e3
        busy += max(0, end - max(start, reach)) / 1e3
        mark = f"  (overlaps {(min(end, reach) - start) / 1e3:.1f} us)" if start < reach else ""
        reach = max(reach, end)
        print(f"{(end - start) / 1e3:9.1f} us  {short(name, 80)}{mark}")
    print(f"{i1 - i0} dispatches, kernel time {total:.1f} us, busy {busy:.1f} us, "
          f"span {(rows[i1][2] - rows[i0][2]) / 1e3:.1f} us")


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    t.add_argument("--top", type=int, default=12)
    c = sub.add_parser("counters")
    c.add_argument("fetch")
    c.add_argument("write")
    c.add_argument("copy_fetch")
    c.add_argument("copy_write")
    c.add_argument("--kernel", default="k_step")
    c.add_argument("--copy-kernel", default="copyBuffer",
                   help="calibration kernel (a 1 GiB copy): the runtime's copyBuffer or the library's k_probe")
    c.add_argument("--nodes", type=int, required=True)
    c.add_argument("--bytes-per-node", type=int, required=True)
    c.add_argument("--tile-width", type=int, required=True, help="tile width of the profiled lattice")
    c.add_argument("--out")
    q = sub.add_parser("sequence")
    q.add_argument("db")
    q.add_argument("--marker", default="k_adam", help="kernel whose consecutive launches bound the sequence")
    args = ap.parse_args(argv)
    {"trace": cmd_trace, "counters": cmd_counters, "sequence": cmd_sequence}[args.cmd](args)


if __name__ == "__main__":
    main()
