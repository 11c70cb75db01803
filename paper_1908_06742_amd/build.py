"""In-tree build of libddf.so for gfx950 with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = [os.path.join(HERE, "csrc", n) for n in ("ddf.hip", "ddf_step_row.hip", "ddf_step_il.hip", "ddf_batch.hip", "ddf_nn.hip", "ddf_probe.hip")]
LIB = os.path.join(HERE, "libddf.so")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # packed FP32 instructions stay off: plain scalar FP32 code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def hipcc():
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.exists(c) or c == "hipcc":
            return c


def _filter(text):
    return "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l)


def build(verbose: bool = True) -> str:
    """Compile every HIP source (in parallel) and link libddf.so (always rebuilds)."""
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(HERE, "csrc", os.path.basename(src) + ".o")
        cmd = [hipcc()] + HIPCC_FLAGS[:] + ["-c", "-o", obj, src]
        cmd.remove("-shared")
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
        objs.append(obj)
    failed = False
    for pr in procs:
        out, _ = pr.communicate()
        if pr.returncode != 0:
            sys.stderr.write(_filter(out) + "\n")
            failed = True
    if failed:
        raise RuntimeError("hipcc failed compiling libddf sources")
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(_filter(r.stdout + r.stderr) + "\n")
        raise RuntimeError("hipcc failed linking libddf.so")
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    build()
