"""Pins of the FP64 U-Net reference: convolution against scipy's correlate2d, pooling
and upsampling against their definitions, and the full backward pass against
central finite differences of the forward pass."""
import numpy as np
import pytest
import torch
from scipy.signal import correlate2d

from oracle import unet as U


def test_conv3x3_matches_correlate2d():
    r = np.random.default_rng(0)
    x = r.standard_normal((2, 7, 9, 3))
    w = r.standard_normal((9, 4, 3))
    b = r.standard_normal(4)
    y = U.conv3x3(x, w, b)
    for n in range(2):
        for co in range(4):
            ref = b[co] + sum(correlate2d(x[n, :, :, ci], w[:, co, ci].reshape(3, 3), mode="same") for ci in range(3))
            assert np.allclose(y[n, :, :, co], ref, atol=1e-12)


def test_pool_and_upsample_definitions():
    r = np.random.default_rng(1)
    x = r.standard_normal((2, 6, 8, 3))
    p = U.pool2(x)
    assert np.allclose(p[1, 2, 3], x[1, 4:6, 6:8].mean(axis=(0, 1)))
    u = U.up2(p)
    assert np.allclose(u[1, 5, 7], p[1, 2, 3]) and u.shape == x.shape
    # the backward functions are the adjoints: <pool(x), y> = <x, pool^T(y)>
    y = r.standard_normal(p.shape)
    assert np.isclose(np.sum(U.pool2(x) * y), np.sum(x * U.pool2_backward(y)))
    z = r.standard_normal(x.shape)
    assert np.isclose(np.sum(U.up2(p) * z), np.sum(p * U.up2_backward(z)))


def test_backward_matches_finite_differences():
    base, levels, cout = 4, 3, 2
    r = np.random.default_rng(2)
    p = U.init_params(base=base, cin=3, cout=cout, levels=levels, seed=3)
    for k in p:
        if k.endswith(".b"):
            p[k] = 0.1 * r.standard_normal(p[k].shape)
    x = r.standard_normal((2, 8, 8, 3))
    R = r.standard_normal((2, 8, 8, cout))

    def loss(pp):
        out, _ = U.forward(pp, x, base=base, levels=levels, cout=cout)
        return float(np.sum(out * R))

    out, cache = U.forward(p, x, base=base, levels=levels, cout=cout)
    g = U.backward(p, cache, R, base=base, levels=levels, cout=cout)
    assert set(g) == set(p)
    eps = 1e-6
    for name in p:
        flat = p[name].reshape(-1)
        for idx in r.choice(flat.size, size=min(3, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + eps
            lp = loss(p)
            flat[idx] = old - eps
            lm = loss(p)
            flat[idx] = old
            fd = (lp - lm) / (2 * eps)
            an = g[name].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (name, idx, fd, an)


def test_mse_gradient():
    # the returned gradient is that of the returned loss: central differences of the
    # loss (a quadratic, so they are exact up to rounding) at every element
    r = np.random.default_rng(4)
    o = r.standard_normal((2, 4, 4, 4))
    t = r.standard_normal((2, 4, 4, 4))
    w = np.array([1.0, 0.5, 2.0, 1.5])
    loss, d = U.mse(o, t, w)
    # the loss is the per-pixel mean of the weighted squared error (a plain loop)
    ref = 0.0
    for n in range(2):
        for i in range(4):
            for j in range(4):
                ref += sum(w[c] * (o[n, i, j, c] - t[n, i, j, c]) ** 2 for c in range(4))
    assert abs(loss - ref / 32.0) < 1e-14
    eps = 1e-4
    fd = np.empty_like(o)
    for idx in np.ndindex(o.shape):
        op, om = o.copy(), o.copy()
        op[idx] += eps
        om[idx] -= eps
        fd[idx] = (U.mse(op, t, w)[0] - U.mse(om, t, w)[0]) / (2.0 * eps)
    assert np.max(np.abs(fd - d)) < 1e-10


def test_bf16_round_matches_torch_conversion():
    r = np.random.default_rng(5)
    x = np.concatenate([r.standard_normal(20000) * 10.0 ** r.integers(-30, 30, 20000),
                        [0.0, -0.0, 1.0, -1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 3.3895313892515355e38, np.inf, -np.inf]])
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    got = U.bf16_round(x)
    assert np.array_equal(got, ref)
    # ties go to even: 1 + 2^-8 is halfway between 1 and 1 + 2^-7
    assert U.bf16_round(1 + 2 ** -8) == 1.0 and U.bf16_round(1 + 3 * 2 ** -8) == 1 + 2 ** -6
    assert np.isnan(U.bf16_round(np.nan))


def test_quantised_reference_is_the_exact_one_with_identity():
    p = U.init_params(base=4, cin=3, cout=2, levels=3, seed=1)
    x = np.random.default_rng(6).standard_normal((1, 8, 8, 3))
    a, _ = U.forward(p, x, base=4, levels=3, cout=2)
    b, cb = U.forward(p, x, base=4, levels=3, cout=2, q=U.bf16_round)
    assert np.array_equal(b, U.bf16_round(b))
    assert 0 < np.linalg.norm(a - b) / np.linalg.norm(a) < 2e-2
