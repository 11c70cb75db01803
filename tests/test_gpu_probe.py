"""The HBM reference kernels (include/ddf_probe.h) move exactly the bytes they claim:
the copy reproduces its source bit for bit, the write pass zeroes its destination and
the read pass leaves every buffer untouched; the step's access pattern without its
collision moves every population where the step of that parity moves it."""
import ctypes as C

import numpy as np
import pytest
import torch

import workloads as W
from paper_1908_06742_amd import Lattice
from paper_1908_06742_amd import _lib as L

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _probe(kind, unroll, nt, src, dst, nbytes):
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    ptr = lambda t: C.c_void_p(t.data_ptr()) if t is not None else None  # noqa: E731
    L.check(L.lib().ddf_bandwidth_probe(kind, unroll, nt, ptr(src), ptr(dst), nbytes, s))


@pytest.mark.parametrize("unroll", [1, 2, 4, 8])
@pytest.mark.parametrize("nt", [0, 1])
def test_probe_passes_move_exactly_their_bytes(unroll, nt):
    print(f"case: bandwidth probe unroll {unroll} nontemporal {nt}", flush=True)
    g = torch.Generator(device=DEV).manual_seed(7 + unroll)
    n = 3 * 256 * unroll * 4 + 20       # a ragged last workgroup
    src = torch.randint(-2**31, 2**31 - 1, (n + 4,), dtype=torch.int32, device=DEV, generator=g)
    dst = torch.full((n + 4,), -7, dtype=torch.int32, device=DEV)
    ref = src.clone()
    _probe(L.PROBE_COPY, unroll, nt, src, dst, 4 * n)
    torch.cuda.synchronize()
    assert torch.equal(dst[:n], src[:n]) and torch.all(dst[n:] == -7)
    _probe(L.PROBE_READ, unroll, nt, src, dst, 4 * n)
    _probe(L.PROBE_READ, unroll, nt, src, None, 4 * n)
    torch.cuda.synchronize()
    assert torch.equal(src, ref) and torch.equal(dst[:n], src[:n])
    _probe(L.PROBE_WRITE, unroll, nt, None, dst, 4 * n)
    torch.cuda.synchronize()
    assert torch.all(dst[:n] == 0) and torch.all(dst[n:] == -7)


OPP = [0, 3, 4, 1, 2, 7, 8, 5, 6]
EX = [0, 1, 0, -1, 0, 1, -1, -1, 1]
EY = [0, 0, 1, 0, -1, 1, 1, -1, -1]
RAW = {"f64": torch.float64, "f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}


@pytest.mark.parametrize("storage,nx,ny,layout,cap", [
    ("f32", 2048, 24, "interleaved", 2),   # x-interleaved rows: the sub-row wrap of the x-shifts
    ("f32", 96, 40, "row", 0),             # padded rows, a ragged last tile
    ("f64", 1024, 8, "interleaved", 1),
    ("f16", 4096, 6, "interleaved", 3),
    ("bf16", 200, 30, "packed", 0),
])
def test_pattern_probe_moves_populations_like_the_step_without_collision(storage, nx, ny, layout, cap):
    print(f"case: pattern probe {storage} {nx}x{ny} {layout} cap {cap}", flush=True)
    lat = Lattice(W.Problem(nx=nx, ny=ny, storage=storage, layout=layout), device=DEV)
    g = torch.Generator().manual_seed(nx + ny)
    f0 = torch.randn((9, ny, nx), generator=g).to(RAW[storage])
    g0 = torch.randn((9, ny, nx), generator=g).to(RAW[storage])
    lat.set_populations(f0, g0, step=0, raw=True)

    def pops():
        f, gg = lat.get_populations(raw=True)
        torch.cuda.synchronize()
        return f.cpu(), gg.cpu()

    bits = {1: torch.int8, 2: torch.int16, 4: torch.int32, 8: torch.int64}[f0.element_size()]

    def same(a, b):    # bit for bit, signed zeros included
        return torch.equal(a.contiguous().view(bits), b.contiguous().view(bits))

    # even: the node's own slots, each population (sign flipped) into the opposite
    # direction's slot; the rest population is rewritten in place
    lat.pattern_probe(0, cap)
    f1, g1 = pops()
    assert same(f1, -f0[OPP]) and same(g1, -g0[OPP])
    lat.pattern_probe(0, cap)
    f1, g1 = pops()
    assert same(f1, f0) and same(g1, g0)
    # odd: from slot opp(a) of x - c_a to slot a of x + c_a; read back as an even-step
    # state, direction a at z holds direction opp(a) of z - 2 c_a
    lat.pattern_probe(1, cap)
    f2, g2 = pops()
    for a in range(9):
        sh = (2 * EY[a], 2 * EX[a])
        assert same(f2[a], -torch.roll(f0[OPP[a]], sh, dims=(0, 1))), a
        assert same(g2[a], -torch.roll(g0[OPP[a]], sh, dims=(0, 1))), a
    lat.pattern_probe(1, cap)
    f2, g2 = pops()
    assert same(f2, f0) and same(g2, g0) and lat.step_count == 0


def _odd_pattern_model(P, px, py):
    """One odd pattern on memory P (9, ny, nx) in the natural slots of an even step: the
    population of direction a loaded for node x (slot opp(a) of x - c_a, or slot a of x
    itself when that link leaves through a wall) is stored negated where the step stores
    direction opp(a)'s (slot a of x + c_a, or slot opp(a) of x at a wall)."""
    ny, nx = P.shape[1:]
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    out = np.empty_like(P)

    def slot(a, sx, sy):
        """slot of direction a read for nodes (xx, yy) from source nodes (sx, sy)"""
        inside = np.ones_like(xx, bool)
        if not px:
            inside &= (sx >= 0) & (sx < nx)
        if not py:
            inside &= (sy >= 0) & (sy < ny)
        plane = np.where(inside, OPP[a], a)
        cy = np.where(inside, sy % ny, yy)
        cx = np.where(inside, sx % nx, xx)
        if a == 0:
            plane, cy, cx = np.zeros_like(xx), yy, xx
        return plane, cy, cx

    for a in range(9):
        lp, ly, lx = slot(a, xx - EX[a], yy - EY[a])
        b = OPP[a]
        sp, sy, sx = slot(b, xx - EX[b], yy - EY[b])
        out[sp, sy, sx] = -P[lp, ly, lx]
    return out


@pytest.mark.parametrize("storage,nx,ny,layout,px,py", [
    ("f32", 40, 24, "row", False, False),            # cavity: walls on all sides, corner links
    ("f64", 64, 20, "row", True, False),             # channel: periodic in x
    ("f32", 2048, 12, "interleaved", False, False),  # x-interleaved rows with walls
])
def test_pattern_probe_with_walls_reflects_where_the_step_does(storage, nx, ny, layout, px, py):
    print(f"case: pattern probe walls {storage} {nx}x{ny} {layout} periodic {px},{py}", flush=True)
    lat = Lattice(W.Problem(nx=nx, ny=ny, storage=storage, layout=layout, periodic_x=px, periodic_y=py), device=DEV)
    g = torch.Generator().manual_seed(nx * ny)
    f0 = torch.randn((9, ny, nx), generator=g).to(RAW[storage])
    g0 = torch.randn((9, ny, nx), generator=g).to(RAW[storage])
    lat.set_populations(f0, g0, step=0, raw=True)
    bits = {4: torch.int32, 8: torch.int64}[f0.element_size()]

    def same(a, b):
        return torch.equal(a.contiguous().view(bits), torch.as_tensor(b).contiguous().view(bits))

    def pops():
        f, gg = lat.get_populations(raw=True)
        torch.cuda.synchronize()
        return f.cpu(), gg.cpu()

    lat.pattern_probe(0, 0)
    f1, g1 = pops()
    assert same(f1, -f0[OPP]) and same(g1, -g0[OPP])
    lat.pattern_probe(0, 0)
    lat.pattern_probe(1, 0)
    f2, g2 = pops()
    assert same(f2, _odd_pattern_model(f0.numpy(), px, py)) and same(g2, _odd_pattern_model(g0.numpy(), px, py))
    lat.pattern_probe(1, 0)
    f2, g2 = pops()
    assert same(f2, f0) and same(g2, g0)


@pytest.mark.parametrize("bx_max", [0, 64])     # flat tiles of 512 nodes; 64-wide rectangular tiles
def test_batch_pattern_probe_matches_the_model_on_every_instance(bx_max):
    from paper_1908_06742_amd.batch import Batch
    print(f"case: batch pattern probe tiles {bx_max}", flush=True)
    probs = [W.cavity_problem(40, 500.0, 0.08, storage="f32"),
             W.Problem(nx=64, ny=20, periodic_x=True, periodic_y=False, storage="f32"),
             W.cavity_problem(37, 900.0, 0.06, storage="f32")]
    b = Batch(probs, device=DEV)
    b.init([W.rest_fields(p.nx, p.ny) for p in probs])
    b.set_tiling(bx_max, 0)
    g = torch.Generator().manual_seed(11 + bx_max)
    views = []
    for i, p in enumerate(probs):
        po, fo = C.c_int64(), C.c_int64()
        L.check(L.lib().ddf_batch_offsets(b._h, i, C.byref(po), C.byref(fo)))
        plane = (p.nx * p.ny + 63) // 64 * 64
        inst = []
        for buf in (b.pop_f, b.pop_g):
            flat = buf[po.value:po.value + 4 * 9 * plane].view(torch.float32)
            inst.append(flat.view(9, plane)[:, :p.nx * p.ny].view(9, p.ny, p.nx))
        views.append(inst)
        for v in inst:
            v.copy_(torch.randn(v.shape, generator=g).to(DEV))
    torch.cuda.synchronize()
    start = [[v.cpu().clone() for v in inst] for inst in views]

    def same(a, b_):
        return torch.equal(a.contiguous().view(torch.int32), torch.as_tensor(b_).contiguous().view(torch.int32))

    b.pattern_probe(0)
    torch.cuda.synchronize()
    for inst, s0 in zip(views, start):
        for v, v0 in zip(inst, s0):
            assert same(v.cpu(), -v0[OPP])
    b.pattern_probe(0)
    b.pattern_probe(1)
    torch.cuda.synchronize()
    for p, inst, s0 in zip(probs, views, start):
        for v, v0 in zip(inst, s0):
            assert same(v.cpu(), _odd_pattern_model(v0.numpy(), p.periodic_x, p.periodic_y))
    b.pattern_probe(1)
    torch.cuda.synchronize()
    for inst, s0 in zip(views, start):
        for v, v0 in zip(inst, s0):
            assert same(v.cpu(), v0)
    assert b.step_count == 0
