"""x-interleaved rows (the layout the library takes for wide lattices that stream from
HBM) and packed rows (the batch's layout) against padded row-major rows and against
the oracle.

A layout only moves populations in memory, so every layout must give the same bits
after any number of steps, in every storage format (stochastic rounding included),
with walls, moving walls, body forces and every scalar model, and extraction must give
the same outputs; reductions agree up to their summation order."""
import math
import sys
import zlib

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from paper_1908_06742_amd import Lattice

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

# the narrowest width each storage allows for x-interleaved rows (a 64-node sub-row
# stride of one 128-byte line)
NX = {"f64": 1024, "f32": 2048, "f16": 4096, "bf16": 4096, "bf16sr": 4096}


# fields compared on a common scale (a component can vanish by symmetry)
GROUPS = (("ux", "uy"), ("Sxx", "Syy", "Sxy", "wz", "dxuy", "dyux"), ("dxphi", "dyphi"), ("Lx", "Ly"))


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _fields(nx, ny, seed, u=0.03):
    r = np.random.default_rng(seed)
    return (1.0 + 0.01 * r.standard_normal((ny, nx)), u * r.standard_normal((ny, nx)),
            u * r.standard_normal((ny, nx)), 1.0 + 0.1 * r.standard_normal((ny, nx)))


def _case(kind, storage, model, nx=None):
    nx = NX[storage] if nx is None else nx
    if kind == "periodic":
        pr = W.Problem(nx=nx, ny=5, storage=storage, scalar_model=model)
    elif kind == "cavity":
        pr = W.cavity_problem(nx, 400.0, 0.08, phi_lid=1.2, phi_walls=1.0, storage=storage).with_(ny=7, scalar_model=model)
    elif kind == "channel":
        pr = W.channel_problem(nx, 6, 0.7, 0.6, force=(2e-5, 1e-6), u_top=0.02).with_(storage=storage, scalar_model=model)
    elif kind == "fourroll":
        pr = W.fourroll_problem(nx, 0.05 * 2.0 * math.pi / nx, 0.03).with_(ny=4, storage=storage, scalar_model=model)
    else:
        raise ValueError(kind)
    return pr, _fields(nx, pr.ny, zlib.crc32(f"{kind}/{storage}".encode()))


def _pair(pr, fields, steps, tile=None):
    row = Lattice(pr.with_(layout="row"), device=DEV)
    il = Lattice(pr.with_(layout="interleaved"), device=DEV)
    assert row.layout == "row" and il.layout == "interleaved"
    if tile:
        il.set_tile_width(tile)
    row.init(*fields).step(steps)
    il.init(*fields).step(steps)
    return row, il


@pytest.mark.parametrize("storage", ["f64", "f32", "f16", "bf16", "bf16sr"])
@pytest.mark.parametrize("kind", ["periodic", "cavity", "channel", "fourroll"])
@pytest.mark.parametrize("steps", [1, 2, 5])
def test_interleaved_rows_step_bit_for_bit(storage, kind, steps):
    model = "central" if kind == "channel" else ("srt" if kind == "fourroll" else "mrt")
    pr, fields = _case(kind, storage, model)
    say(f"case: layout {kind} {storage} {model} steps={steps} ({pr.nx}x{pr.ny})")
    row, il = _pair(pr, fields, steps)
    fr, gr = row.get_populations(raw=True)
    fi, gi = il.get_populations(raw=True)
    torch.cuda.synchronize()
    assert torch.equal(fr.view(torch.int8), fi.view(torch.int8))
    assert torch.equal(gr.view(torch.int8), gi.view(torch.int8))
    # extraction: the same formulas in another kernel, where the compiler may contract
    # other products into fused multiply-adds; equal to the rounding of the compute type
    tol = 1e-13 if storage == "f64" else 2e-6
    for dt in (torch.float64, torch.float32):
        er, ei = row.extract(dtype=dt), il.extract(dtype=dt)
        for k in er:
            a, b = er[k], ei[k]
            assert torch.equal(torch.isnan(a), torch.isnan(b)), k
            m = ~torch.isnan(a)
            grp = next((g for g in GROUPS if k in g), (k,))
            scale = max(float(er[j][~torch.isnan(er[j])].abs().max()) for j in grp)
            if scale > 0:
                assert float((a[m] - b[m]).abs().max()) <= tol * scale, (k, dt)
    sr, si = row.reduce(), il.reduce()
    for k in ("mass", "scalar", "umax", "phimin", "nonfinite"):
        assert abs(sr[k] - si[k]) <= 1e-14 * max(1.0, abs(sr[k])), k


def test_interleaved_rows_any_tile_width_and_graph_runs():
    pr, fields = _case("cavity", "f32", "mrt")
    ref = Lattice(pr.with_(layout="row"), device=DEV).init(*fields).step(203)
    fr, _ = ref.get_populations(raw=True)
    for tile in (64, 128, 256, 512):
        say(f"case: layout tile {tile}")
        il = Lattice(pr.with_(layout="interleaved"), device=DEV)
        il.set_tile_width(tile).set_workgroups_per_cu(2, 2).init(*fields).step(203)   # two graph replays + 3 eager
        fi, _ = il.get_populations(raw=True)
        torch.cuda.synchronize()
        assert torch.equal(fr.view(torch.int8), fi.view(torch.int8)), tile


def test_interleaved_rows_checkpoint_round_trip():
    # raw populations written by one layout and read back by the other continue the same run
    pr, fields = _case("channel", "bf16sr", "mrt")
    row, il = _pair(pr, fields, 3)
    f, g = row.get_populations(raw=True)
    il2 = Lattice(pr.with_(layout="interleaved"), device=DEV).set_populations(f, g, step=3, raw=True)
    row.step(4)
    il2.step(4)
    a, b = row.get_populations(raw=True), il2.get_populations(raw=True)
    torch.cuda.synchronize()
    assert all(torch.equal(x.view(torch.int16), y.view(torch.int16)) for x, y in zip(a, b))
    # absolute FP64 populations too
    f64, g64 = row.get_populations()
    il3 = Lattice(pr.with_(layout="interleaved"), device=DEV).set_populations(f64, g64, step=7)
    row3 = Lattice(pr.with_(layout="row"), device=DEV).set_populations(f64, g64, step=7)
    il3.step(2)
    row3.step(2)
    a, b = row3.get_populations(raw=True), il3.get_populations(raw=True)
    torch.cuda.synchronize()
    assert all(torch.equal(x.view(torch.int16), y.view(torch.int16)) for x, y in zip(a, b))


@pytest.mark.parametrize("kind", ["cavity", "fourroll"])
@pytest.mark.parametrize("steps", [6, 7])
def test_interleaved_rows_match_the_oracle(kind, steps):
    pr, fields = _case(kind, "f64", "mrt")
    say(f"case: layout oracle {kind} steps={steps}")
    il = Lattice(pr.with_(layout="interleaved"), device=DEV).init(*fields).step(steps)
    out = {k: v.cpu().numpy() for k, v in il.extract().items()}
    f, g = (t.cpu().numpy() for t in il.get_populations())
    o = oracle.Oracle(pr, nthreads=8)
    fo, go, ref = o.run(fields, steps)
    for a, b in ((f, fo), (g, go)):
        assert np.max(np.abs(a - b)) / np.max(np.abs(b)) < 1e-12
    for k in ("rho", "ux", "uy", "phi"):
        sc = np.max(np.abs(ref[k])) if k not in ("ux", "uy") else max(np.max(np.abs(ref["ux"])), np.max(np.abs(ref["uy"])))
        assert np.max(np.abs(out[k] - ref[k])) / sc < 1e-12, k
    m = np.isfinite(ref["wz"])
    assert np.array_equal(m, np.isfinite(out["wz"]))
    sc = max(np.max(np.abs(ref[k][m])) for k in ("Sxx", "Syy", "Sxy", "wz"))
    for k in ("Sxx", "Syy", "Sxy", "wz"):
        assert np.max(np.abs(out[k][m] - ref[k][m])) / sc < 1e-10, k


def _compare(row, other, storage):
    fr, gr = row.get_populations(raw=True)
    fo, go = other.get_populations(raw=True)
    torch.cuda.synchronize()
    assert torch.equal(fr.view(torch.int8), fo.view(torch.int8))
    assert torch.equal(gr.view(torch.int8), go.view(torch.int8))
    tol = 1e-13 if storage == "f64" else 2e-6
    for dt in (torch.float64, torch.float32):
        er, eo = row.extract(dtype=dt), other.extract(dtype=dt)
        for k in er:
            a, b = er[k], eo[k]
            assert torch.equal(torch.isnan(a), torch.isnan(b)), k
            m = ~torch.isnan(a)
            grp = next((g for g in GROUPS if k in g), (k,))
            scale = max(float(er[j][~torch.isnan(er[j])].abs().max()) for j in grp)
            if scale > 0:
                assert float((a[m] - b[m]).abs().max()) <= tol * scale, (k, dt)
    sr, so = row.reduce(), other.reduce()
    for k in ("mass", "scalar", "umax", "phimin", "nonfinite"):
        assert abs(sr[k] - so[k]) <= 1e-14 * max(1.0, abs(sr[k])), k


# widths that leave rows ending inside a 128-byte line (and one that fills whole lines)
@pytest.mark.parametrize("storage", ["f64", "f32", "f16", "bf16", "bf16sr"])
@pytest.mark.parametrize("kind,nx", [("periodic", 77), ("cavity", 131), ("channel", 45), ("fourroll", 64)])
@pytest.mark.parametrize("steps", [1, 2, 5])
def test_packed_rows_step_bit_for_bit(storage, kind, nx, steps):
    model = "central" if kind == "channel" else ("srt" if kind == "fourroll" else "mrt")
    pr, fields = _case(kind, storage, model, nx=nx)
    say(f"case: packed {kind} {storage} {model} steps={steps} ({pr.nx}x{pr.ny})")
    row = Lattice(pr.with_(layout="row"), device=DEV)
    pk = Lattice(pr.with_(layout="packed"), device=DEV)
    assert row.layout == "row" and pk.layout == "packed"
    assert pk.pitch == pr.nx and row.pitch % 64 == 0
    row.init(*fields).step(steps)
    pk.init(*fields).step(steps)
    _compare(row, pk, storage)


def test_packed_rows_checkpoint_round_trip_and_tiles():
    # raw populations written by one layout and read back by the other continue the same
    # run (stochastic rounding: the keys name slots of padded rows in every layout)
    pr, fields = _case("channel", "bf16sr", "mrt", nx=45)
    row = Lattice(pr.with_(layout="row"), device=DEV).init(*fields).step(3)
    f, g = row.get_populations(raw=True)
    pk = Lattice(pr.with_(layout="packed"), device=DEV).set_populations(f, g, step=3, raw=True)
    row.step(4)
    pk.step(4)
    _compare(row, pk, "bf16sr")
    pr, fields = _case("cavity", "f32", "mrt", nx=131)
    ref = Lattice(pr.with_(layout="row"), device=DEV).init(*fields).step(203)
    fr, _ = ref.get_populations(raw=True)
    for tile in (64, 128, 256, 512):
        say(f"case: packed tile {tile}")
        pk = Lattice(pr.with_(layout="packed"), device=DEV).set_tile_width(tile).init(*fields).step(203)
        fp, _ = pk.get_populations(raw=True)
        torch.cuda.synchronize()
        assert torch.equal(fr.view(torch.int8), fp.view(torch.int8)), tile


@pytest.mark.parametrize("steps", [6, 7])
def test_packed_rows_match_the_oracle(steps):
    pr, fields = _case("cavity", "f64", "mrt", nx=131)
    say(f"case: packed oracle steps={steps}")
    pk = Lattice(pr.with_(layout="packed"), device=DEV).init(*fields).step(steps)
    f, g = (t.cpu().numpy() for t in pk.get_populations())
    fo, go, _ = oracle.Oracle(pr, nthreads=8).run(fields, steps)
    for a, b in ((f, fo), (g, go)):
        assert np.max(np.abs(a - b)) / np.max(np.abs(b)) < 1e-12
