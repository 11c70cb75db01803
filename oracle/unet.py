"""FP64 NumPy reference of the surrogate U-Net (forward and backward).

TEST INFRASTRUCTURE ONLY (the GPU surrogate never imports it).  The network is not
part of the paper's method; this reference pins the GPU kernels' arithmetic:
3x3 convolutions with zero padding (cross-correlation, as in the GPU kernels), ReLU,
2x2 average pooling, nearest 2x upsampling, channel concatenation and a weighted MSE.
Tensors are NHWC float64; weights w[9][Cout][Cin] with tap = 3 ky + kx.

Pins (tests/test_oracle_unet.py): the convolution against scipy.signal.correlate2d,
pooling and upsampling against reshape/repeat definitions, every backward against
central finite differences of the forward, and the BF16 rounding against torch's
CPU conversion.

`forward` and `backward` take an optional quantiser `q` applied wherever a network
that stores activations and activation gradients in a 16-bit format rounds them:
each layer output (after ReLU), each pooled tensor, the loss gradient, each data
gradient, each upsampling adjoint and each skip-gradient sum.  With `q=bf16_round`
the reference follows a BF16-storage network's arithmetic up to accumulation order;
with the default it is the exact FP64 network.
"""
from __future__ import annotations

import numpy as np


def bf16_round(x):
    """Nearest bfloat16 value (ties to even) of float32(x), returned as float64.
    bfloat16 keeps the top 16 bits of the IEEE binary32 pattern."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    bits = f.view(np.uint32).astype(np.uint64)
    keep_nan = np.isnan(f)
    bits = (bits + 0x7FFF + ((bits >> 16) & 1)) & 0xFFFF0000
    out = bits.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(keep_nan, np.nan, out)


def _ident(x):
    return x


def conv3x3(x, w, b=None):
    """y[n, i, j, co] = b[co] + sum_{ky, kx, ci} x[n, i + ky - 1, j + kx - 1, ci] w[3 ky + kx, co, ci]."""
    N, H, W, Ci = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    y = np.zeros((N, H, W, w.shape[1]))
    for tap in range(9):
        ky, kx = divmod(tap, 3)
        y += np.tensordot(xp[:, ky:ky + H, kx:kx + W, :], w[tap].T, axes=([3], [0]))
    if b is not None:
        y += b
    return y


def conv3x3_backward(x, w, dy):
    """Gradients of conv3x3 w.r.t. x, w and b."""
    N, H, W, Ci = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for tap in range(9):
        ky, kx = divmod(tap, 3)
        patch = xp[:, ky:ky + H, kx:kx + W, :]
        dw[tap] = np.tensordot(dy, patch, axes=([0, 1, 2], [0, 1, 2]))
        dxp[:, ky:ky + H, kx:kx + W, :] += np.tensordot(dy, w[tap], axes=([3], [0]))
    return dxp[:, 1:-1, 1:-1, :], dw, dy.sum(axis=(0, 1, 2))


def pool2(x):
    N, H, W, C = x.shape
    return x.reshape(N, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def pool2_backward(dy):
    return np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2) / 4.0


def up2(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up2_backward(dy):
    N, H, W, C = dy.shape
    return dy.reshape(N, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


def mse(out4, target, weights):
    """Weighted squared error per pixel, loss = (1/npix) sum_p sum_c w_c (out - t)^2, and
    its gradient with respect to out, 2 w_c (out - t) / npix (one objective for both)."""
    d = out4 - target
    npix = d.shape[0] * d.shape[1] * d.shape[2]
    loss = float(np.sum(weights * d * d)) / npix
    return loss, 2.0 * weights * d / npix


# Layer table of the 4-level U-Net with base width `base`: (name, cin, cout, relu).
def layers(base=32, cin=3, cout=4, levels=4):
    ch = [base * 2 ** k for k in range(levels)]
    out = []
    prev = cin
    for k in range(levels):
        out.append((f"enc{k}a", prev, ch[k], True))
        out.append((f"enc{k}b", ch[k], ch[k], True))
        prev = ch[k]
    for k in range(levels - 2, -1, -1):
        out.append((f"dec{k}a", prev + ch[k], ch[k], True))
        out.append((f"dec{k}b", ch[k], ch[k], True))
        prev = ch[k]
    out.append(("head", prev, cout, False))
    return out


def init_params(base=32, cin=3, cout=4, levels=4, seed=0):
    """He-normal weights, zero biases (float64)."""
    r = np.random.default_rng(seed)
    p = {}
    for name, ci, co, _ in layers(base, cin, cout, levels):
        p[name + ".w"] = r.standard_normal((9, co, ci)) * np.sqrt(2.0 / (9 * ci))
        p[name + ".b"] = np.zeros(co)
    return p


def forward(p, x, base=32, levels=4, cout=4, q=_ident):
    """Returns the output and the cache the backward pass needs."""
    L = {name: (ci, co, relu) for name, ci, co, relu in layers(base, x.shape[3], cout, levels)}
    cache = {}

    def conv(name, inp):
        y = conv3x3(inp, p[name + ".w"], p[name + ".b"])
        if L[name][2]:
            y = np.maximum(y, 0.0)
        y = q(y)
        cache[name] = (inp, y)
        return y

    h = x
    skips = []
    for k in range(levels):
        if k > 0:
            h = q(pool2(h))
        h = conv(f"enc{k}a", h)
        h = conv(f"enc{k}b", h)
        skips.append(h)
    for k in range(levels - 2, -1, -1):
        h = np.concatenate([up2(h), skips[k]], axis=3)
        h = conv(f"dec{k}a", h)
        h = conv(f"dec{k}b", h)
    out = conv("head", h)
    return out, cache


def backward(p, cache, dout, base=32, levels=4, cout=4, q=_ident):
    """Gradients of every parameter for the upstream gradient dout (already rounded
    by the caller when q rounds)."""
    cin = cache["enc0a"][0].shape[3]
    L = {name: (ci, co, relu) for name, ci, co, relu in layers(base, cin, cout, levels)}
    g = {}

    def conv_back(name, dy):
        inp, y = cache[name]
        if L[name][2]:
            dy = dy * (y > 0)
        dx, dw, db = conv3x3_backward(inp, p[name + ".w"], dy)
        g[name + ".w"] = dw
        g[name + ".b"] = db
        return q(dx)

    ch = [base * 2 ** k for k in range(levels)]
    dh = conv_back("head", dout)
    dskip = [None] * levels
    for k in range(levels - 1):
        dh = conv_back(f"dec{k}b", dh)
        dh = conv_back(f"dec{k}a", dh)
        cu = dh.shape[3] - ch[k]
        dskip[k] = dh[..., cu:]
        dh = q(up2_backward(dh[..., :cu]))
    # bottleneck and encoder
    for k in range(levels - 1, -1, -1):
        if dskip[k] is not None:
            dh = q(dh + dskip[k])
        dh = conv_back(f"enc{k}b", dh)
        dh = conv_back(f"enc{k}a", dh)
        if k > 0:
            dh = pool2_backward(dh)
    return g
