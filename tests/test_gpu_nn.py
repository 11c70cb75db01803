"""GPU tests of the surrogate-network kernels against the FP64 NumPy reference
(oracle/unet.py), fed with the same BF16-rounded inputs and weights.

Bars: a kernel that stores BF16 rounds its FP32 accumulation once, so every stored
element of a convolution, data gradient, pooling or MSE gradient must lie within one
BF16 ulp of the BF16-rounded FP64 reference, widened only by the FP32 accumulation bound
(terms x 2^-24 x the sum of the absolute terms) where the result cancels; weight and
bias gradients accumulate in FP32 from BF16 operands and are compared at 1e-3.  The whole network is compared with a reference that rounds to BF16
where the kernels store (oracle/unet.py's quantiser): what is left is FP32 against FP64
accumulation order flipping an occasional BF16 rounding.  The output is bounded at 5e-3
(and within 3e-2 of the exact FP64 network).  Gradients are checked twice: the
reference backward at the GPU's own forward state (same ReLU masks) at 1e-2 per layer
and 5e-3 for the whole vector, and the independent reference end to end, where a
flipped mask near zero moves deep-layer gradients, at 6e-2 and 2e-2."""
import ctypes as C
import re as re_mod

import numpy as np
import pytest
import torch

from oracle import unet as U
from paper_1908_06742_amd import _lib as L
from paper_1908_06742_amd.surrogate import UNet

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def p(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def bf(a):
    """numpy -> bf16 device tensor, and the rounded values back as float64."""
    t = torch.tensor(np.asarray(a, np.float32)).to(torch.bfloat16).to(DEV).contiguous()
    return t, t.float().cpu().numpy().astype(np.float64)


def np_of(t, shape):
    return t.float().cpu().numpy().astype(np.float64).reshape(shape)


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-30))


def s0():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def bf16_ulp(v):
    """Spacing of bfloat16 values (8 significant bits) at |v|."""
    a = np.maximum(np.abs(np.asarray(v, np.float64)), 2.0 ** -126)
    return 2.0 ** (np.floor(np.log2(a)) - 7)


def assert_bf16_ulp(got, ref, mag, nterms):
    """got: values a kernel stored in BF16 after accumulating nterms terms in FP32; ref:
    the exact result; mag: the sum of the terms' magnitudes.  Each stored value must be
    within one BF16 ulp of the BF16-rounded reference, plus the FP32 accumulation error
    bound nterms * 2^-24 * mag (which matters only where the sum cancels)."""
    got = np.asarray(got, np.float64)
    q = U.bf16_round(np.asarray(ref, np.float64))
    tol = bf16_ulp(q) + nterms * 2.0 ** -24 * np.asarray(mag, np.float64)
    err = np.abs(got - q)
    assert np.all(err <= tol), (int(np.sum(err > tol)), float(np.max(err / tol)))


@pytest.mark.parametrize("B,H,W,Cin,Cout", [(2, 8, 16, 32, 64), (1, 16, 16, 48, 32), (1, 4, 8, 16, 32)])
@pytest.mark.parametrize("relu", [0, 1])
def test_conv3x3_forward(B, H, W, Cin, Cout, relu):
    r = np.random.default_rng(Cin + Cout + relu)
    xt, x = bf(r.standard_normal((B, H, W, Cin)))
    w = r.standard_normal((9, Cout, Cin)) / np.sqrt(9 * Cin)
    wft, wq = bf(w)
    b = r.standard_normal(Cout).astype(np.float32)
    bt = torch.tensor(b, device=DEV)
    out = torch.zeros(B * H * W * Cout, dtype=torch.bfloat16, device=DEV)
    L.check(L.lib().ddf_nn_conv3x3(p(xt), B, H, W, Cin, Cin, 0, p(wft), p(bt), p(out), Cout, Cout, 0, relu, 0, None, 0, 0, s0()))
    ref = U.conv3x3(x, wq.reshape(9, Cout, Cin), b.astype(np.float64))
    mag = U.conv3x3(np.abs(x), np.abs(wq).reshape(9, Cout, Cin), np.abs(b).astype(np.float64))
    if relu:
        ref = np.maximum(ref, 0)
    assert_bf16_ulp(np_of(out, ref.shape), ref, mag, 9 * Cin + 1)


def test_conv3x3_slices_and_accumulate():
    B, H, W, Cin, Cout = 1, 8, 8, 32, 32
    r = np.random.default_rng(5)
    # input is channels [16, 48) of a 64-channel tensor; output goes to channels [32, 64) of a 96-channel one
    big, bigq = bf(r.standard_normal((B, H, W, 64)))
    wt, wq = bf(r.standard_normal((9, Cout, Cin)) / 17)
    out0, out0q = bf(r.standard_normal((B, H, W, 96)))
    L.check(L.lib().ddf_nn_conv3x3(p(big), B, H, W, Cin, 64, 16, p(wt), None, p(out0), Cout, 96, 32, 0, 1, None, 0, 0, s0()))
    ref = out0q.copy()
    ref[..., 32:64] += U.conv3x3(bigq[..., 16:48], wq.reshape(9, Cout, Cin))
    mag = np.abs(out0q[..., 32:64]) + U.conv3x3(np.abs(bigq[..., 16:48]), np.abs(wq).reshape(9, Cout, Cin))
    got = np_of(out0, ref.shape)
    assert_bf16_ulp(got[..., 32:64], ref[..., 32:64], mag, 9 * Cin + 1)
    assert np.array_equal(got[..., :32], out0q[..., :32]) and np.array_equal(got[..., 64:], out0q[..., 64:])


def test_conv3x3_data_and_weight_gradients():
    B, H, W, Cin, Cout = 2, 8, 16, 32, 64
    r = np.random.default_rng(7)
    xt, x = bf(r.standard_normal((B, H, W, Cin)))
    w = (r.standard_normal((9, Cout, Cin)) / np.sqrt(9 * Cin)).astype(np.float32)
    wmaster = torch.tensor(w, device=DEV)
    wf = torch.empty(9 * Cout * Cin, dtype=torch.bfloat16, device=DEV)
    wd = torch.empty_like(wf)
    L.check(L.lib().ddf_nn_cast_weights(p(wmaster), Cout, Cin, Cout, Cin, p(wf), p(wd), s0()))
    wq = np_of(wf, (9, Cout, Cin))
    dyt, dy = bf(r.standard_normal((B, H, W, Cout)))
    dx = torch.zeros(B * H * W * Cin, dtype=torch.bfloat16, device=DEV)
    L.check(L.lib().ddf_nn_conv3x3(p(dyt), B, H, W, Cout, Cout, 0, p(wd), None, p(dx), Cin, Cin, 0, 0, 0, None, 0, 0, s0()))
    rdx, rdw, rdb = U.conv3x3_backward(x, wq, dy)
    mdx = U.conv3x3_backward(np.abs(x), np.abs(wq), np.abs(dy))[0]
    assert_bf16_ulp(np_of(dx, rdx.shape), rdx, mdx, 9 * Cout)
    ws = torch.empty(L.lib().ddf_nn_wgrad_workspace_bytes(B, H, W, Cin, Cout, None), dtype=torch.uint8, device=DEV)
    dw = torch.zeros(9 * Cout * Cin, dtype=torch.float32, device=DEV)
    db = torch.zeros(Cout, dtype=torch.float32, device=DEV)
    L.check(L.lib().ddf_nn_conv3x3_wgrad(p(xt), B, H, W, Cin, Cin, 0, p(dyt), Cout, Cout, p(dw), p(db), 0, p(ws), s0()))
    assert rel(dw.cpu().numpy().reshape(9, Cout, Cin), rdw) < 1e-3
    assert rel(db.cpu().numpy(), rdb) < 1e-3


def test_pool_up_slice_relu_kernels():
    r = np.random.default_rng(9)
    B, H, W, C = 2, 8, 8, 16
    xt, x = bf(r.standard_normal((B, H, W, C)))
    pooled = torch.empty(B * H * W * C // 4, dtype=torch.bfloat16, device=DEV)
    L.check(L.lib().ddf_nn_pool2(p(xt), B, H, W, C, C, 0, p(pooled), s0()))
    assert_bf16_ulp(np_of(pooled, (B, H // 2, W // 2, C)), U.pool2(x), U.pool2(np.abs(x)), 4)
    up = torch.zeros(B * H * W * 24, dtype=torch.bfloat16, device=DEV)
    L.check(L.lib().ddf_nn_up2(p(pooled), B, H // 2, W // 2, C, p(up), 24, 8, s0()))
    pq = np_of(pooled, (B, H // 2, W // 2, C))
    assert np.array_equal(np_of(up, (B, H, W, 24))[..., 8:24], U.up2(pq))
    gt, g = bf(r.standard_normal((B, H, W, 24)))
    din = torch.empty(B * H * W * C // 4, dtype=torch.bfloat16, device=DEV)
    L.check(L.lib().ddf_nn_up2_bwd(p(gt), B, H // 2, W // 2, C, 24, 8, p(din), s0()))
    assert_bf16_ulp(np_of(din, pq.shape), U.up2_backward(g[..., 8:24]), U.up2_backward(np.abs(g[..., 8:24])), 4)
    dp = torch.zeros(B * H * W * C, dtype=torch.bfloat16, device=DEV)
    L.check(L.lib().ddf_nn_pool2_bwd(p(din), B, H, W, C, p(dp), C, 0, None, 0, s0()))
    dq = np_of(din, pq.shape)
    assert_bf16_ulp(np_of(dp, x.shape), U.pool2_backward(dq), U.pool2_backward(np.abs(dq)), 1)
    dst = torch.zeros(B * H * W * 40, dtype=torch.bfloat16, device=DEV)
    L.check(L.lib().ddf_nn_slice(p(xt), C, 0, p(dst), 40, 24, B * H * W, C, 0, s0()))
    assert np.array_equal(np_of(dst, (B, H, W, 40))[..., 24:40], x)
    gg = xt.clone()
    L.check(L.lib().ddf_nn_relu_bwd(p(gg), p(xt), gg.numel(), s0()))
    assert np.array_equal(np_of(gg, x.shape), np.where(x > 0, x, 0.0))


@pytest.mark.parametrize("shapes", [
    # padded to multiples of 32 (32 x 32 tiles through LDS), one without the data-gradient copy
    [(32, 5, 32, 32, True), (64, 32, 64, 32, True), (96, 40, 96, 64, False), (256, 256, 256, 256, True),
     (384, 128, 384, 128, True)],
    # other padded sizes (one element per thread)
    [(10, 5, 12, 8, True), (64, 32, 64, 32, True), (3, 7, 3, 9, False)],
])
def test_cast_weights_multi_matches_per_layer_casts(shapes):
    r = np.random.default_rng(7)
    layers, ref = [], []
    for co, ci, cop, cip, with_wd in shapes:
        w = torch.tensor(r.standard_normal(9 * co * ci), dtype=torch.float32, device=DEV)
        bufs = [torch.full((9 * cop * cip,), 3.0, dtype=torch.bfloat16, device=DEV) for _ in range(4)]
        wd1, wd2 = (bufs[1], bufs[3]) if with_wd else (None, None)
        L.check(L.lib().ddf_nn_cast_weights(p(w), co, ci, cop, cip, p(bufs[0]), p(wd1) if wd1 is not None else None,
                                            s0()))
        layers.append(L.CastLayer(w.data_ptr(), bufs[2].data_ptr(), wd2.data_ptr() if wd2 is not None else None,
                                  co, ci, cop, cip))
        ref.append((w, bufs, with_wd))
    arr = (L.CastLayer * len(layers))(*layers)
    L.check(L.lib().ddf_nn_cast_weights_multi(len(layers), arr, s0()))
    torch.cuda.synchronize()
    for (co, ci, cop, cip, with_wd), (w, bufs, _) in zip(shapes, ref):
        assert torch.equal(bufs[0], bufs[2])
        assert torch.equal(bufs[1], bufs[3])
        if not with_wd:
            assert torch.all(bufs[3].float() == 3.0)
        wf = bufs[2].float().cpu().numpy().reshape(9, cop, cip)
        assert np.all(wf[:, co:, :] == 0) and np.all(wf[:, :, ci:] == 0)


@pytest.mark.parametrize("accumulate", [0, 1])
@pytest.mark.parametrize("W,Cout,Cin", [
    (64, 32, 64),      # k_conv3x3<4, 1>
    (128, 32, 32),     # row streaming, 32 output channels per workgroup
    (64, 64, 64),      # row streaming, two 32-channel tiles per workgroup, two rows
    (128, 64, 32),     # row streaming, two tiles, four rows
    (64, 128, 128),    # row streaming, four tiles per workgroup
    (32, 256, 64),     # row streaming at width 32
    (16, 64, 32),      # LDS-staged kernel, 64-pixel rows not available: k_conv3x3<2, 2>
])
def test_masked_data_gradient_and_pool_adjoint_equal_relu_backward_after(W, Cout, Cin, accumulate):
    # masking each contribution (the fused path of the network's backward) gives the bits
    # of the unmasked kernel followed by the ReLU adjoint, when what is accumulated into
    # is already masked
    r = np.random.default_rng(31 + accumulate + W + Cout)
    B, H, cs = 2, 8, Cout + 32
    dyt, _ = bf(r.standard_normal((B, H, W, Cin)))
    wd, _ = bf(0.1 * r.standard_normal((9, Cout, Cin)))
    act, _ = bf(r.standard_normal((B, H, W, cs)))              # mask channels [16, 16 + Cout) of a wider tensor
    old = torch.where(act[..., 16:16 + Cout] > 0, torch.tensor(r.standard_normal((B, H, W, Cout)), dtype=torch.bfloat16,
                                                                device=DEV), torch.zeros((), dtype=torch.bfloat16, device=DEV))
    fused = old.clone().contiguous()
    ref = old.clone().contiguous()
    L.check(L.lib().ddf_nn_conv3x3(p(dyt), B, H, W, Cin, Cin, 0, p(wd), None, p(fused), Cout, Cout, 0, 0, accumulate,
                                   p(act), cs, 16, s0()))
    L.check(L.lib().ddf_nn_conv3x3(p(dyt), B, H, W, Cin, Cin, 0, p(wd), None, p(ref), Cout, Cout, 0, 0, accumulate,
                                   None, 0, 0, s0()))
    mask = act[..., 16:16 + Cout].contiguous()
    L.check(L.lib().ddf_nn_relu_bwd(p(ref), p(mask), ref.numel(), s0()))
    torch.cuda.synchronize()
    assert torch.equal(fused, ref)
    assert (fused != 0).any()
    # pooling adjoint, masked per child
    C = 32
    d, _ = bf(r.standard_normal((B, H // 2, W // 2, C)))
    a, _ = bf(r.standard_normal((B, H, W, C)))
    o = torch.where(a > 0, torch.tensor(r.standard_normal((B, H, W, C)), dtype=torch.bfloat16, device=DEV),
                    torch.zeros((), dtype=torch.bfloat16, device=DEV))
    for vec in (True, False):
        fused = o.clone().contiguous()
        ref = o.clone().contiguous()
        Cp = C if vec else C - 3          # C % 8 != 0 takes the single-element kernel
        L.check(L.lib().ddf_nn_pool2_bwd(p(d), B, H, W, Cp, p(fused), Cp, 0, p(a), accumulate, s0()))
        L.check(L.lib().ddf_nn_pool2_bwd(p(d), B, H, W, Cp, p(ref), Cp, 0, None, accumulate, s0()))
        n = B * H * W * Cp
        L.check(L.lib().ddf_nn_relu_bwd(p(ref), p(a), n, s0()))
        torch.cuda.synchronize()
        assert torch.equal(fused.reshape(-1)[:n], ref.reshape(-1)[:n]), vec


@pytest.mark.parametrize("C,cs,co", [(16, 32, 8), (12, 20, 4), (32, 96, 64)])   # 16-byte and single-element forms
@pytest.mark.parametrize("accumulate", [0, 1])
def test_pool_reads_and_adjoint_writes_channel_slices(C, cs, co, accumulate):
    # pooling of channels [co, co + C) of a wider tensor, and the adjoint (masked by a
    # tensor of the same layout) into that slice, leaving the other channels as they were:
    # a skip connection held inside the decoder's concatenation buffer
    r = np.random.default_rng(C + cs + co + accumulate)
    B, H, W = 2, 6, 8
    xt, x = bf(r.standard_normal((B, H, W, cs)))
    pooled = torch.empty(B * H * W * C // 4, dtype=torch.bfloat16, device=DEV)
    L.check(L.lib().ddf_nn_pool2(p(xt), B, H, W, C, cs, co, p(pooled), s0()))
    xs = x[..., co:co + C]
    assert_bf16_ulp(np_of(pooled, (B, H // 2, W // 2, C)), U.pool2(xs), U.pool2(np.abs(xs)), 4)
    dt, dq = bf(r.standard_normal((B, H // 2, W // 2, C)))
    mt, mq = bf(r.standard_normal((B, H, W, cs)))
    gt, g0 = bf(r.standard_normal((B, H, W, cs)))
    L.check(L.lib().ddf_nn_pool2_bwd(p(dt), B, H, W, C, p(gt), cs, co, p(mt), accumulate, s0()))
    got = np_of(gt, (B, H, W, cs))
    want = np.where(mq[..., co:co + C] > 0, U.pool2_backward(dq), 0.0)
    mag = np.abs(want)
    if accumulate:
        want = want + g0[..., co:co + C]
        mag = mag + np.abs(g0[..., co:co + C])
    assert_bf16_ulp(got[..., co:co + C], want, mag, 1)
    keep = np.ones(cs, bool)
    keep[co:co + C] = False
    assert np.array_equal(got[..., keep], g0[..., keep])


@pytest.mark.parametrize("B,H,W,C,cs,co", [
    (2, 6, 40, 24, 40, 8),      # C / 8 = 3: lanes find their pixel by division
    (3, 4, 72, 64, 96, 32),     # 576 lanes per full-resolution row: three blocks, the last one ragged
    (1, 2, 520, 8, 8, 0),       # one channel group, 520 pixels per row
])
def test_resampling_kernels_on_multi_block_rows(B, H, W, C, cs, co):
    # the 16-byte pooling and upsampling kernels and their adjoints run on a grid of
    # pixel rows (several blocks per row): slices of a wider tensor, against the oracle
    r = np.random.default_rng(B * 1000 + W)
    xt, x = bf(r.standard_normal((B, H, W, cs)))
    pooled = torch.empty(B * H * W * C // 4, dtype=torch.bfloat16, device=DEV)
    L.check(L.lib().ddf_nn_pool2(p(xt), B, H, W, C, cs, co, p(pooled), s0()))
    xs = x[..., co:co + C]
    assert_bf16_ulp(np_of(pooled, (B, H // 2, W // 2, C)), U.pool2(xs), U.pool2(np.abs(xs)), 4)
    pq = np_of(pooled, (B, H // 2, W // 2, C))
    mt, mq = bf(r.standard_normal((B, H, W, cs)))
    gt, g0 = bf(r.standard_normal((B, H, W, cs)))
    L.check(L.lib().ddf_nn_pool2_bwd(p(pooled), B, H, W, C, p(gt), cs, co, p(mt), 1, s0()))
    got = np_of(gt, (B, H, W, cs))
    want = np.where(mq[..., co:co + C] > 0, U.pool2_backward(pq), 0.0)
    assert_bf16_ulp(got[..., co:co + C], want + g0[..., co:co + C], np.abs(want) + np.abs(g0[..., co:co + C]), 1)
    keep = np.ones(cs, bool)
    keep[co:co + C] = False
    assert np.array_equal(got[..., keep], g0[..., keep])
    up = torch.zeros(B * H * W * cs, dtype=torch.bfloat16, device=DEV)
    L.check(L.lib().ddf_nn_up2(p(pooled), B, H // 2, W // 2, C, p(up), cs, co, s0()))
    ug = np_of(up, (B, H, W, cs))
    assert np.array_equal(ug[..., co:co + C], U.up2(pq)) and not np.any(ug[..., keep])
    ht, hq = bf(r.standard_normal((B, H, W, cs)))
    din = torch.empty(B * H * W * C // 4, dtype=torch.bfloat16, device=DEV)
    L.check(L.lib().ddf_nn_up2_bwd(p(ht), B, H // 2, W // 2, C, cs, co, p(din), s0()))
    hs = hq[..., co:co + C]
    assert_bf16_ulp(np_of(din, pq.shape), U.up2_backward(hs), U.up2_backward(np.abs(hs)), 4)


def test_pool_rejects_strides_that_miss_the_channels():
    x = torch.zeros(2 * 4 * 4 * 16, dtype=torch.bfloat16, device=DEV)
    o = torch.zeros(2 * 2 * 2 * 16, dtype=torch.bfloat16, device=DEV)
    assert L.lib().ddf_nn_pool2(p(x), 2, 4, 4, 16, 16, 8, p(o), s0()) == L.DDF_ERR_ARG
    assert L.lib().ddf_nn_pool2_bwd(p(o), 2, 4, 4, 16, p(x), 8, 0, None, 0, s0()) == L.DDF_ERR_ARG


def test_mse_and_adam():
    r = np.random.default_rng(11)
    npix = 4 * 16 * 16
    ot, o = bf(r.standard_normal((npix, 32)))
    t = r.standard_normal((npix, 4)).astype(np.float32)
    tt = torch.tensor(t, device=DEV)
    wts = (C.c_float * 4)(1.0, 0.5, 2.0, 1.5)
    dout = torch.empty_like(ot)
    loss = torch.zeros(1, dtype=torch.float64, device=DEV)
    ws = torch.empty(L.lib().ddf_nn_mse_workspace_bytes(npix), dtype=torch.uint8, device=DEV)
    L.check(L.lib().ddf_nn_mse(p(ot), 32, p(tt), npix, wts, p(dout), p(loss), p(ws), s0()))
    rl, rg = U.mse(o[:, :4].reshape(1, 1, npix, 4), t.astype(np.float64).reshape(1, 1, npix, 4),
                   np.array([1.0, 0.5, 2.0, 1.5]))
    rg = rg.reshape(npix, 4)
    assert abs(loss.item() - rl) / rl < 1e-6
    d = np_of(dout, (npix, 32))
    assert_bf16_ulp(d[:, :4], rg, np.abs(rg), 4)
    assert np.all(d[:, 4:] == 0)
    n = 1000
    w = r.standard_normal(n).astype(np.float32)
    g = r.standard_normal(n).astype(np.float32)
    tw, tg = torch.tensor(w, device=DEV), torch.tensor(g, device=DEV)
    tm, tv = torch.zeros_like(tw), torch.zeros_like(tw)
    for step in (1, 2):
        L.check(L.lib().ddf_nn_adam(p(tw), p(tg), p(tm), p(tv), n, 1e-3, 0.9, 0.999, 1e-8, step, 0.0, s0()))
    m = v = 0.0
    ww = w.astype(np.float64)
    for step in (1, 2):
        m = 0.9 * m + 0.1 * g
        v = 0.999 * v + 0.001 * g * g
        ww = ww - 1e-3 * (m / (1 - 0.9 ** step)) / (np.sqrt(v / (1 - 0.999 ** step)) + 1e-8)
    assert np.max(np.abs(tw.cpu().numpy() - ww)) < 1e-6


@pytest.mark.parametrize("levels,H", [(3, 32), (4, 32)])
def test_unet_forward_backward_against_reference(levels, H):
    B, W = 2, H
    net = UNet(base=32, levels=levels, device=DEV, seed=1)
    r = np.random.default_rng(13)
    prm = net.params_numpy()
    for k in prm:
        if k.endswith(".b"):
            prm[k] = 0.05 * r.standard_normal(prm[k].shape)
    net.set_params_numpy(prm)
    re = torch.tensor([150.0, 2500.0], device=DEV)
    u = torch.tensor([0.06, 0.09], device=DEV)
    net.inputs(re, u, H, W)
    x = np_of(net.x, (B, H, W, 32))[..., :5]
    out = net.forward(B, H, W)
    # the reference uses the BF16-rounded weights the GPU actually multiplies
    pq = {}
    for name, ci, co, _ in net.table:
        cip, cop = net._pdims(name, ci, co)
        pq[name + ".w"] = np_of(net.wf[name], (9, cop, cip))[:, :co, :ci]
        pq[name + ".b"] = prm[name + ".b"]
    # the BF16-storage reference rounds where the kernels round: differences left are
    # accumulation order (FP32 on the matrix cores against FP64), which flips an
    # occasional BF16 rounding
    q = U.bf16_round
    ref, cache = U.forward(pq, x, base=32, levels=levels, cout=4, q=q)
    got = np_of(out, (B, H, W, 32))[..., :4]
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 5e-3
    exact, _ = U.forward(pq, x, base=32, levels=levels, cout=4)
    assert np.linalg.norm(got - exact) / np.linalg.norm(exact) < 3e-2
    target = r.standard_normal((B, H, W, 4)).astype(np.float32)
    tt = torch.tensor(target, device=DEV).reshape(-1)
    net.loss_and_grad(tt, B, H, W)
    net.backward(B, H, W)
    _, dref = U.mse(ref, target.astype(np.float64), np.ones(4))
    gg = net.grads_numpy()

    def compare(gref, per_layer, whole):
        errs = {k: np.linalg.norm(gg[k] - gref[k]) / max(np.linalg.norm(gref[k]), 1e-30) for k in gref}
        print("largest per-layer gradient errors:", sorted(errs.items(), key=lambda kv: -kv[1])[:4])
        for name, e in errs.items():
            assert e < per_layer, (name, e)
        a = np.concatenate([gg[k].ravel() for k in sorted(gref)])
        b = np.concatenate([gref[k].ravel() for k in sorted(gref)])
        assert np.linalg.norm(a - b) / np.linalg.norm(b) < whole

    # (1) backward of the reference at the GPU's own forward state (same activations,
    # hence the same ReLU masks): only the backward's accumulation order differs
    def level(key):
        return int(re_mod.search(r"\d", key).group())

    A = {k: np_of(v, (B, H >> level(k), W >> level(k), -1)) for k, v in net.A.items() if k != "head"}

    def output_of(name):
        # an encoder output other than the deepest one lives in its decoder's concatenation
        k = int(name[3])
        if name.startswith("enc") and name[4] == "b" and k < levels - 1:
            return A[f"cat{k}"][..., net.ch[k + 1]:net.ch[k + 1] + net.ch[k]]
        return A[name]

    gcache = {}
    for name, ci, co, _ in net.table:
        if name == "head":
            gcache[name] = (A["dec0b"], got)
            continue
        k, part = int(name[3]), name[4]
        if name.startswith("enc"):
            src = (x if k == 0 else A[f"pool{k}"]) if part == "a" else A[f"enc{k}a"]
        else:
            src = A[f"cat{k}"] if part == "a" else A[f"dec{k}a"]
        gcache[name] = (src[..., :ci], output_of(name)[..., :co])
    _, dgpu = U.mse(got, target.astype(np.float64), np.ones(4))
    compare(U.backward(pq, gcache, q(dgpu), base=32, levels=levels, cout=4, q=q), 1e-2, 5e-3)
    # (2) the independent BF16-storage reference end to end: ReLU masks of activations
    # near zero may differ, which moves the deepest layers' gradients by a few percent
    compare(U.backward(pq, cache, q(dref), base=32, levels=levels, cout=4, q=q), 6e-2, 2e-2)


def test_training_reduces_loss():
    torch.manual_seed(0)
    B, H, W = 4, 32, 32
    net = UNet(base=32, levels=4, device=DEV, seed=2)
    re = torch.tensor([120.0, 600.0, 1800.0, 4000.0], device=DEV)
    u = torch.tensor([0.05, 0.07, 0.08, 0.1], device=DEV)
    yy, xx = torch.meshgrid(torch.linspace(0, 1, H, device=DEV), torch.linspace(0, 1, W, device=DEV), indexing="ij")
    tgt = torch.stack([torch.stack([torch.sin(3 * xx) * yy * (k + 1) / 4, xx * yy, 0.1 * yy, yy * yy], dim=-1)
                       for k in range(B)]).float().reshape(-1)
    losses = []
    for it in range(60):
        losses.append(net.train_step(re, u, tgt, H, W, lr=2e-3).item())
    assert losses[-1] < 0.2 * losses[0], (losses[0], losses[-1])


@pytest.mark.parametrize("B,H", [(2, 128), (8, 256)])
def test_weight_gradients_on_a_side_stream_match_one_stream(B, H):
    # the weight gradients overlap the data-gradient chain on a second stream; the
    # kernels are the same, so three training steps (Adam and the next forward wait
    # for them) must give bit-identical gradients and weights
    W = H
    user = torch.cuda.Stream(device=DEV)     # a caller's own stream as the network's main stream
    nets = [UNet(base=32, levels=4, device=DEV, seed=5, overlap_wgrad=ov, stream=st)
            for ov, st in ((False, None), (True, None), (True, user))]
    g = torch.Generator(device=DEV).manual_seed(B)
    re = 100.0 + 4900.0 * torch.rand(B, device=DEV, generator=g)
    u = 0.05 + 0.05 * torch.rand(B, device=DEV, generator=g)
    tgt = torch.randn(B * H * W * 4, device=DEV, generator=g)
    torch.cuda.synchronize()
    for it in range(3):
        losses = []
        for net in nets:
            if net.stream is None:
                losses.append(net.train_step(re, u, tgt, H, W, lr=1e-3).item())
            else:
                with torch.cuda.stream(net.stream):
                    loss = net.train_step(re, u, tgt, H, W, lr=1e-3)
                net.stream.synchronize()
                losses.append(loss.item())
        assert losses[0] == losses[1] == losses[2], (it, losses)
        for net in nets[1:]:
            assert torch.equal(nets[0].g, net.g), it
            assert torch.equal(nets[0].w, net.w), it
    assert nets[1]._side is not None and nets[0]._side is None


@pytest.mark.parametrize("C,off", [(32, 0), (13, 0), (32, 2)])   # 16-byte stores; single stores (C % 8, unaligned)
def test_cavity_input_channels(C, off):
    B, H, W = 2, 16, 24
    re = torch.tensor([100.0, 5000.0], device=DEV)
    u = torch.tensor([0.05, 0.1], device=DEV)
    buf = torch.full((off + B * H * W * C,), 7.0, dtype=torch.bfloat16, device=DEV)
    x = buf[off:]
    L.check(L.lib().ddf_nn_cavity_inputs(p(re), p(u), B, H, W, C, 100.0, 5000.0, 0.1, p(x), s0()))
    a = np_of(x, (B, H, W, C))
    assert np.all(np_of(buf[:off], (off,)) == 7.0)
    yy, xx = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    mask = np.where((xx == 0) | (xx == W - 1) | (yy == 0), 1.0, 0.0)
    mask[H - 1, :] = 2.0
    for n in range(B):
        assert np.array_equal(a[n, ..., 0], mask)
        assert np.allclose(a[n, ..., 1], [0.0, 1.0][n], atol=4e-3)
        assert np.allclose(a[n, ..., 2], [0.5, 1.0][n], atol=4e-3)
        assert np.allclose(a[n, ..., 3], xx / (W - 1), atol=4e-3)
        assert np.allclose(a[n, ..., 4], yy / (H - 1), atol=4e-3)
        assert np.all(a[n, ..., 5:] == 0)
    bad = L.lib().ddf_nn_cavity_inputs(p(re), p(u), B, H, W, 4, 100.0, 5000.0, 0.1, p(x), s0())
    assert bad == L.DDF_ERR_ARG


@pytest.mark.parametrize("B,H,W,Cin,Cout", [
    (1, 4, 64, 64, 64),      # row streaming, 64-pixel columns, one strip (small image)
    (1, 3, 128, 96, 32),     # row streaming, 128-pixel columns, 96 input channels
    (1, 1, 64, 32, 32),      # row streaming, a single row: both neighbour rows are padding
    (3, 37, 192, 64, 96),    # row streaming, 64-pixel columns, 3 x 6 tiles, ragged strips
    (1, 3, 64, 32, 256),     # row streaming, the most output channels (8 output tiles)
    (1, 2, 128, 256, 32),    # row streaming, 8 input tiles, the bias from the first only
    (2, 5, 32, 32, 64),      # 32-pixel blocks, single tiles
    (1, 2, 16, 128, 256),    # 16-pixel blocks, single tiles over 4 x 8 tile groups
    (1, 129, 256, 32, 64),   # row streaming, strips of 8 rows, the last one of a single row
    (2, 17, 1024, 64, 128),  # row streaming, 8 columns per image, 2 x 4 tiles
    (1, 1040, 32, 32, 64),   # 32-pixel blocks, two output tiles
    (2, 4, 8, 32, 32),       # rows of 8: the gather kernel
])
def test_weight_gradient_kernels(B, H, W, Cin, Cout):
    r = np.random.default_rng(B * 1000 + H * 100 + W + Cin + Cout)
    # input taken as channels [16, 16 + Cin) of a wider tensor
    cs = Cin + 32
    xt, x = bf(r.standard_normal((B, H, W, cs)))
    dyt, dy = bf(r.standard_normal((B, H, W, Cout)))
    _, rdw, rdb = U.conv3x3_backward(x[..., 16:16 + Cin], np.zeros((9, Cout, Cin)), dy)
    ws = torch.empty(L.lib().ddf_nn_wgrad_workspace_bytes(B, H, W, Cin, Cout, None), dtype=torch.uint8, device=DEV)
    dw = torch.full((9 * Cout * Cin,), 0.5, dtype=torch.float32, device=DEV)
    db = torch.full((Cout,), 0.25, dtype=torch.float32, device=DEV)
    L.check(L.lib().ddf_nn_conv3x3_wgrad(p(xt), B, H, W, Cin, cs, 16, p(dyt), Cout, Cout, p(dw), p(db), 1, p(ws), s0()))
    assert rel(dw.cpu().numpy().reshape(9, Cout, Cin) - 0.5, rdw) < 1e-5
    assert rel(db.cpu().numpy() - 0.25, rdb) < 1e-5
    # deterministic: the same call gives the same bits
    dw2 = torch.zeros_like(dw)
    db2 = torch.zeros_like(db)
    L.check(L.lib().ddf_nn_conv3x3_wgrad(p(xt), B, H, W, Cin, cs, 16, p(dyt), Cout, Cout, p(dw2), p(db2), 0, p(ws), s0()))
    dw3 = torch.zeros_like(dw)
    L.check(L.lib().ddf_nn_conv3x3_wgrad(p(xt), B, H, W, Cin, cs, 16, p(dyt), Cout, Cout, p(dw3), None, 0, p(ws), s0()))
    assert torch.equal(dw2, dw3)


def test_elementwise_kernels_with_unaligned_channel_counts():
    # 12 channels: the one-element-per-thread forms of pooling, upsampling and slices
    r = np.random.default_rng(21)
    B, H, W, C = 2, 6, 8, 12
    xt, x = bf(r.standard_normal((B, H, W, C)))
    pooled = torch.empty(B * H * W * C // 4, dtype=torch.bfloat16, device=DEV)
    L.check(L.lib().ddf_nn_pool2(p(xt), B, H, W, C, C, 0, p(pooled), s0()))
    pq = np_of(pooled, (B, H // 2, W // 2, C))
    assert_bf16_ulp(pq, U.pool2(x), U.pool2(np.abs(x)), 4)
    up = torch.zeros(B * H * W * 20, dtype=torch.bfloat16, device=DEV)
    L.check(L.lib().ddf_nn_up2(p(pooled), B, H // 2, W // 2, C, p(up), 20, 4, s0()))
    assert np.array_equal(np_of(up, (B, H, W, 20))[..., 4:16], U.up2(pq))
    gt, g = bf(r.standard_normal((B, H, W, 20)))
    din = torch.empty(B * H * W * C // 4, dtype=torch.bfloat16, device=DEV)
    L.check(L.lib().ddf_nn_up2_bwd(p(gt), B, H // 2, W // 2, C, 20, 4, p(din), s0()))
    assert_bf16_ulp(np_of(din, pq.shape), U.up2_backward(g[..., 4:16]), U.up2_backward(np.abs(g[..., 4:16])), 4)
    dp = torch.zeros(B * H * W * C, dtype=torch.bfloat16, device=DEV)
    L.check(L.lib().ddf_nn_pool2_bwd(p(din), B, H, W, C, p(dp), C, 0, None, 0, s0()))
    dq = np_of(din, pq.shape)
    assert_bf16_ulp(np_of(dp, x.shape), U.pool2_backward(dq), U.pool2_backward(np.abs(dq)), 1)
    dst, dq = bf(r.standard_normal((B, H, W, 20)))
    L.check(L.lib().ddf_nn_slice(p(xt), C, 0, p(dst), 20, 3, B * H * W, C, 1, s0()))
    want = dq.copy()
    want[..., 3:15] += x
    assert_bf16_ulp(np_of(dst, (B, H, W, 20))[..., 3:15], want[..., 3:15], np.abs(dq[..., 3:15]) + np.abs(x), 2)
    gg = xt.clone()
    L.check(L.lib().ddf_nn_relu_bwd(p(gg), p(xt), gg.numel() - 3, s0()))
    got = np_of(gg, x.shape).reshape(-1)
    ref = np.where(x > 0, x, 0.0).reshape(-1)
    assert np.array_equal(got[:-3], ref[:-3]) and np.array_equal(got[-3:], x.reshape(-1)[-3:])


@pytest.mark.parametrize("B,H,W,Cin,Cout,cs_in,co_in,cs_out,co_out,acc", [
    (1, 3, 64, 64, 128, 64, 0, 128, 0, 0),       # 64-pixel segments, 4 channel tiles
    (2, 2, 128, 32, 64, 64, 16, 96, 32, 1),      # 64-pixel segments, 2 tiles, slices, accumulate
    (1, 4, 32, 96, 128, 96, 0, 128, 0, 0),       # 32-pixel segments, 4 tiles
    (1, 3, 256, 64, 32, 64, 0, 64, 32, 1),       # 128-pixel segments, 1 tile, slices, accumulate
    (1, 2, 512, 32, 96, 32, 0, 96, 0, 0),        # 128-pixel segments, 3 channel tiles
    (2, 3, 256, 32, 32, 64, 16, 64, 32, 1),      # 32 -> 32 channels: 256-pixel segments, slices, accumulate
    (1, 2, 512, 32, 32, 32, 0, 32, 0, 0),        # 32 -> 32 channels: 256-pixel segments
    (1, 8, 128, 32, 32, 32, 0, 32, 0, 0),        # 32 output channels, rows a multiple of 4: row streaming
    (2, 4, 256, 96, 32, 96, 0, 64, 32, 1),       # row streaming, 3 input chunks, slices, accumulate
    (1, 12, 128, 128, 32, 160, 16, 32, 0, 0),    # row streaming, 4 input chunks, input slice
    (1, 4, 128, 32, 64, 32, 0, 64, 0, 0),        # row streaming, 64 channels: 64-pixel rows, 2 tiles per workgroup
    (1, 4, 128, 128, 64, 160, 32, 96, 16, 1),    # row streaming, 128-pixel rows, 2 tiles, slices, accumulate
    (1, 8, 128, 64, 192, 64, 0, 192, 0, 0),      # row streaming, 192 channels: 3 workgroup columns
    (2, 4, 64, 128, 128, 128, 0, 128, 0, 0),     # row streaming at width 64, 4 tiles per workgroup
    (1, 6, 64, 160, 384, 160, 0, 384, 0, 1),     # 5 input chunks, 384 channels, accumulate
    (1, 2, 64, 128, 64, 128, 0, 64, 0, 0),       # row streaming at width 64, 2 tiles
    (2, 4, 32, 256, 256, 288, 32, 256, 0, 0),    # row streaming at width 32, 8 input chunks, input slice
    (1, 3, 64, 128, 128, 128, 0, 128, 0, 0),     # odd row count: the LDS-staged kernel
])
def test_conv3x3_lds_configs(B, H, W, Cin, Cout, cs_in, co_in, cs_out, co_out, acc):
    r = np.random.default_rng(B + H + W + Cin + Cout)
    xt, x = bf(r.standard_normal((B, H, W, cs_in)))
    wt, wq = bf(r.standard_normal((9, Cout, Cin)) / np.sqrt(9 * Cin))
    b = r.standard_normal(Cout).astype(np.float32)
    bt = torch.tensor(b, device=DEV)
    out0, out0q = bf(r.standard_normal((B, H, W, cs_out)))
    L.check(L.lib().ddf_nn_conv3x3(p(xt), B, H, W, Cin, cs_in, co_in, p(wt), p(bt), p(out0), Cout, cs_out, co_out, 1,
                                   acc, None, 0, 0, s0()))
    ref = np.maximum(U.conv3x3(x[..., co_in:co_in + Cin], wq.reshape(9, Cout, Cin), b.astype(np.float64)), 0)
    mag = U.conv3x3(np.abs(x[..., co_in:co_in + Cin]), np.abs(wq).reshape(9, Cout, Cin), np.abs(b).astype(np.float64))
    if acc:
        ref = ref + out0q[..., co_out:co_out + Cout]
        mag = mag + np.abs(out0q[..., co_out:co_out + Cout])
    got = np_of(out0, (B, H, W, cs_out))
    assert_bf16_ulp(got[..., co_out:co_out + Cout], ref, mag, 9 * Cin + 2)
    untouched = np.ones(cs_out, bool)
    untouched[co_out:co_out + Cout] = False
    assert np.array_equal(got[..., untouched], out0q[..., untouched])


@pytest.mark.parametrize("W,Cin,d_cs,d_co", [
    (128, 32, 96, 64),    # 128-pixel columns: the skip slice of a level-0 concatenation gradient
    (192, 64, 160, 32),   # 64-pixel columns, two input tiles, a slice in the middle
])
def test_row_streaming_weight_gradient_of_channel_slices(W, Cin, d_cs, d_co):
    # The surrogate's weight gradients read the output gradient as a channel slice of a
    # wider buffer (offset through the pointer, stride d_cs) and the input as a slice too;
    # against the float64 sums over all pixels, with accumulation into dw and db.
    B, H, Cout = 2, 19, 32
    r = np.random.default_rng(W + Cin + d_co)
    cs = Cin + 16
    xt, x = bf(r.standard_normal((B, H, W, cs)))
    dyt, dy = bf(r.standard_normal((B, H, W, d_cs)))
    xs_, d2 = x[..., 8:8 + Cin], dy[..., d_co:d_co + Cout]
    _, rdw, rdb = U.conv3x3_backward(xs_, np.zeros((9, Cout, Cin)), d2)
    ws = torch.empty(L.lib().ddf_nn_wgrad_workspace_bytes(B, H, W, Cin, Cout, None), dtype=torch.uint8, device=DEV)
    dw = torch.full((9 * Cout * Cin,), -1.0, dtype=torch.float32, device=DEV)
    db = torch.full((Cout,), 2.0, dtype=torch.float32, device=DEV)
    dptr = C.c_void_p(dyt.data_ptr() + 2 * d_co)
    L.check(L.lib().ddf_nn_conv3x3_wgrad(p(xt), B, H, W, Cin, cs, 8, dptr, Cout, d_cs, p(dw), p(db), 1, p(ws), s0()))
    assert rel(dw.cpu().numpy().reshape(9, Cout, Cin) + 1.0, rdw) < 1e-5
    assert rel(db.cpu().numpy() - 2.0, rdb) < 1e-5


def test_row_streaming_weight_gradient_with_ragged_strips():
    # 64 -> 32 channels on 2 x 683 x 192 pixels: three 64-pixel columns per image, strips of
    # 32 rows, the last one of each column 11 rows long.  Every entry against the float64
    # sum over all pixels.
    B, H, W, Cin, Cout = 2, 683, 192, 64, 32
    r = np.random.default_rng(77)
    xt, x = bf(r.standard_normal((B, H, W, Cin)))
    dyt, dy = bf(r.standard_normal((B, H, W, Cout)))
    chunk = C.c_int32()
    nbytes = L.lib().ddf_nn_wgrad_workspace_bytes(B, H, W, Cin, Cout, C.byref(chunk))
    rows = chunk.value // 64
    assert chunk.value % 64 == 0 and H % rows == 11
    assert nbytes == B * 3 * (H // rows + 1) * (9 * Cout * Cin + Cout) * 4
    ws = torch.empty(nbytes, dtype=torch.uint8, device=DEV)
    dw = torch.empty(9 * Cout * Cin, dtype=torch.float32, device=DEV)
    db = torch.empty(Cout, dtype=torch.float32, device=DEV)
    L.check(L.lib().ddf_nn_conv3x3_wgrad(p(xt), B, H, W, Cin, Cin, 0, p(dyt), Cout, Cout, p(dw), p(db), 0, p(ws), s0()))
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    d2 = dy.reshape(-1, Cout)
    ref = np.empty((9, Cout, Cin))
    mag = np.empty((9, Cout, Cin))
    for tap in range(9):
        ky, kx = divmod(tap, 3)
        xs = xp[:, ky:ky + H, kx:kx + W, :].reshape(-1, Cin)
        ref[tap] = d2.T @ xs
        mag[tap] = np.abs(d2).T @ np.abs(xs)
    got = dw.cpu().numpy().reshape(9, Cout, Cin)
    assert np.max(np.abs(got - ref) / mag) < 2e-5     # FP32 sums of exact BF16 products
    gb = db.cpu().numpy()
    assert np.max(np.abs(gb - d2.sum(axis=0)) / np.abs(d2).sum(axis=0)) < 2e-5


@pytest.mark.parametrize("H,Cin,Cout", [
    (256, 32, 32),     # 32 -> 32 at 256^2: 256-pixel convolution segments, row-streaming weight gradient
    (256, 96, 32),     # the level-0 decoder input: 128-pixel segments
    (128, 64, 64),     # 64-pixel segments x 2 channel tiles; weight gradient over 2 x 2 tiles
    (64, 384, 128),    # the level-2 decoder input: 4 channel tiles
    (128, 192, 64),    # the level-1 decoder input
    (32, 256, 256),    # the bottom level: 32-pixel segments
])
def test_full_size_layers_sampled_outputs(H, Cin, Cout):
    # The surrogate's layer shapes at the training batch (8 x H x H): forward and data
    # gradient at sampled pixels, computed by the reference on each sample's 3 x 3
    # neighbourhood (all a centre output depends on), and sampled weight-gradient entries
    # as plain sums over all pixels.
    B, W = 8, H
    r = np.random.default_rng(H + Cin + Cout)
    xt, x = bf(r.standard_normal((B, H, W, Cin)))
    dyt, dy = bf(r.standard_normal((B, H, W, Cout)))
    wmaster = torch.tensor((r.standard_normal((9, Cout, Cin)) / np.sqrt(9 * Cin)).astype(np.float32), device=DEV)
    wf = torch.empty(9 * Cout * Cin, dtype=torch.bfloat16, device=DEV)
    wd = torch.empty_like(wf)
    L.check(L.lib().ddf_nn_cast_weights(p(wmaster), Cout, Cin, Cout, Cin, p(wf), p(wd), s0()))
    wq = np_of(wf, (9, Cout, Cin))
    y = torch.empty(B * H * W * Cout, dtype=torch.bfloat16, device=DEV)
    dx = torch.empty(B * H * W * Cin, dtype=torch.bfloat16, device=DEV)
    L.check(L.lib().ddf_nn_conv3x3(p(xt), B, H, W, Cin, Cin, 0, p(wf), None, p(y), Cout, Cout, 0, 0, 0, None, 0, 0, s0()))
    L.check(L.lib().ddf_nn_conv3x3(p(dyt), B, H, W, Cout, Cout, 0, p(wd), None, p(dx), Cin, Cin, 0, 0, 0, None, 0, 0,
                                   s0()))
    ws = torch.empty(L.lib().ddf_nn_wgrad_workspace_bytes(B, H, W, Cin, Cout, None), dtype=torch.uint8, device=DEV)
    dw = torch.empty(9 * Cout * Cin, dtype=torch.float32, device=DEV)
    db = torch.empty(Cout, dtype=torch.float32, device=DEV)
    L.check(L.lib().ddf_nn_conv3x3_wgrad(p(xt), B, H, W, Cin, Cin, 0, p(dyt), Cout, Cout, p(dw), p(db), 0, p(ws), s0()))
    yg, dxg = np_of(y, (B, H, W, Cout)), np_of(dx, (B, H, W, Cin))
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    dyp = np.pad(dy, ((0, 0), (1, 1), (1, 1), (0, 0)))
    pix = [(0, 0, 0), (B - 1, H - 1, W - 1), (1, 0, W - 1)] + \
          [(int(r.integers(B)), int(r.integers(H)), int(r.integers(W))) for _ in range(40)]
    got_y, ref_y, mag_y, got_dx, ref_dx, mag_dx = [], [], [], [], [], []
    aw = np.abs(wq)
    for n, i, j in pix:
        ref_y.append(U.conv3x3(xp[n:n + 1, i:i + 3, j:j + 3, :], wq)[0, 1, 1])
        mag_y.append(U.conv3x3(np.abs(xp[n:n + 1, i:i + 3, j:j + 3, :]), aw)[0, 1, 1])
        got_y.append(yg[n, i, j])
        ref_dx.append(U.conv3x3_backward(np.zeros((1, 3, 3, Cin)), wq, dyp[n:n + 1, i:i + 3, j:j + 3, :])[0][0, 1, 1])
        mag_dx.append(U.conv3x3_backward(np.zeros((1, 3, 3, Cin)), aw, np.abs(dyp[n:n + 1, i:i + 3, j:j + 3, :]))[0][0, 1, 1])
        got_dx.append(dxg[n, i, j])
    assert_bf16_ulp(np.array(got_y), np.array(ref_y), np.array(mag_y), 9 * Cin)
    assert_bf16_ulp(np.array(got_dx), np.array(ref_dx), np.array(mag_dx), 9 * Cout)
    dwg, dbg = dw.cpu().numpy().reshape(9, Cout, Cin), db.cpu().numpy()
    ent = [(int(r.integers(9)), int(r.integers(Cout)), int(r.integers(Cin))) for _ in range(12)]
    got_w = np.array([dwg[t, co, ci] for t, co, ci in ent])
    ref_w = np.array([np.sum(dy[..., co] * xp[:, t // 3:t // 3 + H, t % 3:t % 3 + W, ci]) for t, co, ci in ent])
    assert rel(got_w, ref_w) < 1e-3
    assert rel(dbg, dy.sum(axis=(0, 1, 2))) < 1e-3
