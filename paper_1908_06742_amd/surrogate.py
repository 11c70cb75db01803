"""Surrogate U-Net for steady lid-driven cavities, on the libddf BF16 MFMA kernels.

Maps (wall mask, Re, lid speed, node coordinates) on an H x W grid to normalised steady fields
(u / U, v / U, (rho - 1) / U^2, phi).  Four levels of two 3x3 convolutions with
ReLU (widths base, 2 base, 4 base, 8 base), 2x2 average pooling down, nearest 2x
upsampling and skip concatenation up, and a 3x3 head.  Activations are NHWC BF16,
accumulation FP32 on the matrix cores, master weights and Adam state FP32.  Every
operation runs in the HIP kernels of include/ddf_nn.h; this module only allocates
buffers (torch) and sequences the calls.

The lattice Boltzmann solver decides convergence: a prediction only initialises the
lattice, and `warm_start_batch` falls back to a cold start for every instance whose
residual after the first check (100 steps) is above 1e-2 or non-finite.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np
import torch

from . import _lib as L

RE_LO, RE_HI, U_REF = 100.0, 5000.0, 0.1
CIN = 5        # mask, log Re, U, x, y
CIN_P = 32     # network input channels (CIN used)
COUT_P = 32    # head output channels (4 used)


def _p(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def layer_table(base=32, levels=4, cin=CIN, cout=4):
    """(name, cin, cout, relu) in forward order."""
    ch = [base * 2 ** k for k in range(levels)]
    out, prev = [], cin
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


def _pad(c):
    return max(32, (c + 31) // 32 * 32)


class UNet:
    def __init__(self, base=32, levels=4, device="cuda", seed=0, stream=None, overlap_wgrad=True):
        self.base, self.levels = base, levels
        self.device = torch.device(device)
        self.stream = stream
        # weight gradients on a second stream, overlapped with the data-gradient chain
        self.overlap_wgrad = overlap_wgrad
        self._side = None
        self.table = layer_table(base, levels)
        self.ch = [base * 2 ** k for k in range(levels)]
        # flat FP32 parameter layout: per layer w[9][cout_p][cin_p] then b[cout_p], channel
        # counts padded to multiples of 32 with zero entries (their gradients are zero, so
        # they stay zero)
        self.off = {}
        n = 0
        for name, ci, co, _ in self.table:
            cip, cop = self._pdims(name, ci, co)
            self.off[name] = (n, n + 9 * cop * cip)
            n += 9 * cop * cip + cop
        self.nparams = n
        r = np.random.default_rng(seed)
        host = np.zeros(n, np.float32)
        for name, ci, co, _ in self.table:
            cip, cop = self._pdims(name, ci, co)
            w0, b0 = self.off[name]
            blk = np.zeros((9, cop, cip), np.float32)
            blk[:, :co, :ci] = r.standard_normal((9, co, ci)) * math.sqrt(2.0 / (9 * ci))
            host[w0:b0] = blk.reshape(-1)
        self.w = torch.tensor(host, device=self.device)
        self.g = torch.zeros_like(self.w)
        self.m = torch.zeros_like(self.w)
        self.v = torch.zeros_like(self.w)
        self.adam_step = 0
        # bf16 copies: forward [9][cout_p][cin_p] and data-gradient [9][cin_p][cout_p]
        self.wf, self.wd = {}, {}
        for name, ci, co, _ in self.table:
            cip, cop = self._pdims(name, ci, co)
            self.wf[name] = torch.empty(9 * cop * cip, dtype=torch.bfloat16, device=self.device)
            self.wd[name] = torch.empty(9 * cip * cop, dtype=torch.bfloat16, device=self.device)
        self.cast()
        self._shape = None

    # ------------------------------------------------------------------ params
    @staticmethod
    def _pdims(name, ci, co):
        return (CIN_P if name == "enc0a" else _pad(ci)), _pad(co)

    def _dims(self, name):
        for nm, ci, co, relu in self.table:
            if nm == name:
                cip, cop = self._pdims(nm, ci, co)
                return ci, co, cip, cop, relu
        raise KeyError(name)

    def _wptr(self, t, name, bias=False):
        w0, b0 = self.off[name]
        return C.c_void_p(t.data_ptr() + 4 * (b0 if bias else w0))

    def _main(self):
        return self.stream if self.stream is not None else torch.cuda.current_stream(self.device)

    def _s(self):
        return C.c_void_p(self._main().cuda_stream)

    def _wgrad_stream(self):
        """Stream of the next weight-gradient launch.  With overlap, the side stream first
        waits for everything queued so far on the main stream (the layer's output gradient
        and, for skip connections, the pooling adjoint accumulated into it); the weight
        gradients run in order on that one stream, so they share the split-K workspace.
        Returns a function that launches on it."""
        if not self.overlap_wgrad:
            s = self._s()
            return lambda launch: launch(s)
        if self._side is None:
            self._side = torch.cuda.Stream(device=self.device)
        ev = torch.cuda.Event()
        ev.record(self._main())
        side = self._side

        def run(launch):
            side.wait_event(ev)
            launch(C.c_void_p(side.cuda_stream))
        return run

    def _join_wgrad(self):
        """The main stream waits for the queued weight gradients (before Adam, and before
        a later forward overwrites the activations they read)."""
        if self.overlap_wgrad and self._side is not None:
            ev = torch.cuda.Event()
            ev.record(self._side)
            self._main().wait_event(ev)

    def cast(self):
        """BF16 forward and data-gradient copies of every layer, one launch per 32 layers."""
        if getattr(self, "_cast_layers", None) is None:
            rows = []
            for name, ci, co, _ in self.table:
                _, _, cip, cop, _ = self._dims(name)
                rows.append(L.CastLayer(self._wptr(self.w, name).value, self.wf[name].data_ptr(),
                                        self.wd[name].data_ptr(), cop, cip, cop, cip))
            self._cast_layers = [(L.CastLayer * len(rows[i:i + L.NN_CAST_MAX_LAYERS]))(*rows[i:i + L.NN_CAST_MAX_LAYERS])
                                 for i in range(0, len(rows), L.NN_CAST_MAX_LAYERS)]
        for arr in self._cast_layers:
            L.check(L.lib().ddf_nn_cast_weights_multi(len(arr), arr, self._s()))

    def state_dict(self):
        return {"w": self.w.detach().cpu().numpy(), "base": self.base, "levels": self.levels}

    def load_state_dict(self, sd):
        assert int(sd["base"]) == self.base and int(sd["levels"]) == self.levels
        self.w.copy_(torch.as_tensor(np.asarray(sd["w"], np.float32), device=self.device))
        self.cast()

    def _unflatten(self, flat):
        h = flat.detach().cpu().numpy().astype(np.float64)
        out = {}
        for name, ci, co, _ in self.table:
            _, _, cip, cop, _ = self._dims(name)
            w0, b0 = self.off[name]
            out[name + ".w"] = h[w0:b0].reshape(9, cop, cip)[:, :co, :ci].copy()
            out[name + ".b"] = h[b0:b0 + co].copy()
        return out

    def params_numpy(self):
        """Parameters as {name.w: [9][cout][cin], name.b: [cout]} float64 arrays (real channels)."""
        return self._unflatten(self.w)

    def grads_numpy(self):
        return self._unflatten(self.g)

    def set_params_numpy(self, p):
        host = self.w.detach().cpu().numpy().copy()
        for name, ci, co, _ in self.table:
            _, _, cip, cop, _ = self._dims(name)
            w0, b0 = self.off[name]
            blk = np.zeros((9, cop, cip), np.float32)
            blk[:, :co, :ci] = p[name + ".w"]
            host[w0:b0] = blk.reshape(-1)
            host[b0:b0 + cop] = 0.0
            host[b0:b0 + co] = p[name + ".b"]
        self.w.copy_(torch.as_tensor(host, device=self.device))
        self.cast()

    # ----------------------------------------------------------------- buffers
    def _alloc(self, B, H, W):
        if self._shape == (B, H, W):
            return
        assert H % (1 << (self.levels - 1)) == 0 and W % (1 << (self.levels - 1)) == 0
        dev, bf = self.device, torch.bfloat16
        A, G = {}, {}

        def t(h, w, c):
            return torch.zeros(B * h * w * c, dtype=bf, device=dev)

        self.x = t(H, W, CIN_P)
        for k in range(self.levels):
            h, w, c = H >> k, W >> k, self.ch[k]
            if k > 0:
                A[f"pool{k}"] = t(h, w, self.ch[k - 1])
            A[f"enc{k}a"] = t(h, w, c)
        # the deepest encoder output is a tensor of its own; every other encoder output (a
        # skip connection) is written straight into the channels [ch[k+1], ch[k+1] + ch[k])
        # of its decoder's concatenation buffer, where the decoder reads it (and its
        # gradient lives in the same channels of the gradient of that buffer)
        k = self.levels - 1
        A[f"enc{k}b"] = t(H >> k, W >> k, self.ch[k])
        for k in range(self.levels - 2, -1, -1):
            h, w = H >> k, W >> k
            A[f"cat{k}"] = t(h, w, self.ch[k + 1] + self.ch[k])
            A[f"dec{k}a"], A[f"dec{k}b"] = t(h, w, self.ch[k]), t(h, w, self.ch[k])
        A["head"] = t(H, W, COUT_P)
        for k, v in A.items():
            G[k] = torch.zeros_like(v)
        self.A, self.G = A, G
        self.ws_bytes = 0
        for name, ci, co, _ in self.table:
            lvl = int(name[3]) if name != "head" else 0
            _, _, cip, cop, _ = self._dims(name)
            self.ws_bytes = max(self.ws_bytes, L.lib().ddf_nn_wgrad_workspace_bytes(B, H >> lvl, W >> lvl, cip, cop, None))
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)
        self.mse_ws = torch.empty(L.lib().ddf_nn_mse_workspace_bytes(B * H * W), dtype=torch.uint8, device=dev)
        self.loss_dev = torch.zeros(1, dtype=torch.float64, device=dev)
        self._shape = (B, H, W)

    # ----------------------------------------------------------------- forward
    def _skip(self, k, grad=False):
        """(tensor, channel stride, channel offset) of encoder output enc{k}b, or of its
        gradient: a tensor of its own at the deepest level, else a channel slice of the
        decoder's concatenation buffer cat{k}."""
        T = self.G if grad else self.A
        if k == self.levels - 1:
            return T[f"enc{k}b"], self.ch[k], 0
        return T[f"cat{k}"], self.ch[k + 1] + self.ch[k], self.ch[k + 1]

    def _conv(self, name, src, src_cs, dst, B, h, w, src_co=0, dst_cs=None, dst_co=0):
        _, _, cip, cop, relu = self._dims(name)
        L.check(L.lib().ddf_nn_conv3x3(_p(src), B, h, w, cip, src_cs, src_co, _p(self.wf[name]),
                                       self._wptr(self.w, name, bias=True), _p(dst), cop,
                                       cop if dst_cs is None else dst_cs, dst_co, int(relu), 0,
                                       None, 0, 0, self._s()))

    def inputs(self, re, u, H, W):
        """Input tensor for per-sample Reynolds numbers and lid speeds (float32 device tensors)."""
        B = re.numel()
        self._alloc(B, H, W)
        L.check(L.lib().ddf_nn_cavity_inputs(_p(re), _p(u), B, H, W, CIN_P, RE_LO, RE_HI, U_REF, _p(self.x), self._s()))
        return self.x

    def forward(self, B, H, W):
        """Runs on self.x (filled by `inputs`); returns the head output [B, H, W, 32] (bf16)."""
        self._alloc(B, H, W)
        lib, s, A = L.lib(), self._s(), self.A
        h = self.x
        hc = CIN_P
        for k in range(self.levels):
            hh, ww = H >> k, W >> k
            if k > 0:
                src, cs, co = self._skip(k - 1)
                L.check(lib.ddf_nn_pool2(_p(src), B, 2 * hh, 2 * ww, self.ch[k - 1], cs, co, _p(A[f"pool{k}"]), s))
                h, hc = A[f"pool{k}"], self.ch[k - 1]
            self._conv(f"enc{k}a", h, hc, A[f"enc{k}a"], B, hh, ww)
            dst, cs, co = self._skip(k)
            self._conv(f"enc{k}b", A[f"enc{k}a"], self.ch[k], dst, B, hh, ww, dst_cs=cs, dst_co=co)
        h, hc = A[f"enc{self.levels - 1}b"], self.ch[self.levels - 1]
        for k in range(self.levels - 2, -1, -1):
            hh, ww = H >> k, W >> k
            ctot = hc + self.ch[k]
            cat = A[f"cat{k}"]
            L.check(lib.ddf_nn_up2(_p(h), B, hh // 2, ww // 2, hc, _p(cat), ctot, 0, s))
            self._conv(f"dec{k}a", cat, ctot, A[f"dec{k}a"], B, hh, ww)
            self._conv(f"dec{k}b", A[f"dec{k}a"], self.ch[k], A[f"dec{k}b"], B, hh, ww)
            h, hc = A[f"dec{k}b"], self.ch[k]
        self._conv("head", h, hc, A["head"], B, H, W)
        return A["head"]

    # ---------------------------------------------------------------- backward
    def _conv_back(self, name, src, src_cs, dsrc, acc, B, h, w, src_relu=True, dy=None):
        """dY (default G[name]; else (tensor, channel stride, offset)) holds the gradient of
        the layer's output, already multiplied by its ReLU's derivative: every producer of a
        gradient masks its contribution with the activation it flows into (here: the data
        gradient, masked with `src` when `src` is a ReLU output)."""
        _, _, cip, cop, relu = self._dims(name)
        lib, s = L.lib(), self._s()
        dyt, dcs, dco = (self.G[name], cop, 0) if dy is None else dy
        # the weight gradient takes the output gradient's channel offset in its pointer
        # (bf16 elements, offsets multiples of 8: 16-byte aligned)
        wgrad = self._wgrad_stream()   # ordered after the producers of dY, before the data gradient
        if dsrc is not None:
            # the data gradient first: the rest of the backward chain waits for it
            mask = _p(src) if src_relu else None
            L.check(lib.ddf_nn_conv3x3(_p(dyt), B, h, w, cop, dcs, dco, _p(self.wd[name]), None, _p(dsrc), cip, cip, 0,
                                       0, int(acc), mask, src_cs, 0, s))
        wgrad(lambda st: L.check(lib.ddf_nn_conv3x3_wgrad(
            _p(src), B, h, w, cip, src_cs, 0, C.c_void_p(dyt.data_ptr() + 2 * dco), cop, dcs, self._wptr(self.g, name),
            self._wptr(self.g, name, bias=True), 0, _p(self.ws), st)))

    def backward(self, B, H, W):
        """Needs G['head'] = dLoss/dOut; fills self.g with every parameter's gradient."""
        lib, s, A, G = L.lib(), self._s(), self.A, self.G
        self._conv_back("head", A["dec0b"], self.ch[0], G["dec0b"], 0, B, H, W)
        for k in range(self.levels - 1):
            hh, ww = H >> k, W >> k
            self._conv_back(f"dec{k}b", A[f"dec{k}a"], self.ch[k], G[f"dec{k}a"], 0, B, hh, ww)
            cu = self.ch[k + 1]
            ctot = cu + self.ch[k]
            self._conv_back(f"dec{k}a", A[f"cat{k}"], ctot, G[f"cat{k}"], 0, B, hh, ww)
            # adjoint of the concatenation: the upsampled part goes to the deeper output; the
            # skip part is already the encoder output's gradient (same channels of G[cat{k}])
            deeper = f"dec{k + 1}b" if k + 1 <= self.levels - 2 else f"enc{self.levels - 1}b"
            L.check(lib.ddf_nn_up2_bwd(_p(G[f"cat{k}"]), B, hh // 2, ww // 2, cu, ctot, 0, _p(G[deeper]), s))
        for k in range(self.levels - 1, -1, -1):
            hh, ww = H >> k, W >> k
            self._conv_back(f"enc{k}b", A[f"enc{k}a"], self.ch[k], G[f"enc{k}a"], 0, B, hh, ww,
                            dy=self._skip(k, grad=True))
            if k > 0:
                # the pooled input is no ReLU output: its gradient is masked per child below
                self._conv_back(f"enc{k}a", A[f"pool{k}"], self.ch[k - 1], G[f"pool{k}"], 0, B, hh, ww,
                                src_relu=False)
                # the pooled input feeds from the previous level's output, which also got a
                # skip gradient: accumulate, masked by that output (same channel layout)
                gk, cs, co = self._skip(k - 1, grad=True)
                ak, _, _ = self._skip(k - 1)
                L.check(lib.ddf_nn_pool2_bwd(_p(G[f"pool{k}"]), B, 2 * hh, 2 * ww, self.ch[k - 1], _p(gk), cs, co,
                                             _p(ak), 1, s))
            else:
                self._conv_back("enc0a", self.x, CIN_P, None, 0, B, hh, ww)
        self._join_wgrad()

    # ---------------------------------------------------------------- training
    def loss_and_grad(self, target, B, H, W, weights=(1.0, 1.0, 1.0, 1.0)):
        """Weighted squared error per pixel of the head output against target (float32
        [B*H*W*4]); sets G['head'] to its gradient and returns the device loss."""
        wts = (C.c_float * 4)(*weights)
        L.check(L.lib().ddf_nn_mse(_p(self.A["head"]), COUT_P, _p(target), B * H * W, wts, _p(self.G["head"]),
                                   _p(self.loss_dev), _p(self.mse_ws), self._s()))
        return self.loss_dev

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
        self.adam_step += 1
        L.check(L.lib().ddf_nn_adam(_p(self.w), _p(self.g), _p(self.m), _p(self.v), self.nparams, lr, beta1, beta2,
                                    eps, self.adam_step, weight_decay, self._s()))
        self.cast()

    def train_step(self, re, u, target, H, W, lr):
        B = re.numel()
        self.inputs(re, u, H, W)
        self.forward(B, H, W)
        loss = self.loss_and_grad(target, B, H, W)
        self.backward(B, H, W)
        self.adam(lr)
        return loss

    # --------------------------------------------------------------- inference
    def predict_fields(self, re, u, H, W):
        """Physical FP64 fields (rho, ux, uy, phi), each [B, H, W], for a warm start."""
        B = re.numel()
        self.inputs(re, u, H, W)
        out = self.forward(B, H, W)
        f = [torch.empty((B, H, W), dtype=torch.float64, device=self.device) for _ in range(4)]
        L.check(L.lib().ddf_nn_cavity_fields(_p(out), COUT_P, _p(u), B, H * W, _p(f[0]), _p(f[1]), _p(f[2]),
                                             _p(f[3]), self._s()))
        return f


def predict_batch_fields(net, re, u, H, W, chunk=16):
    """Network prediction for every (re[i], u[i]) as concatenated FP64 device fields
    (rho, ux, uy, phi), each [N, H, W], evaluated `chunk` samples at a time."""
    N = re.numel()
    out = [torch.empty((N, H, W), dtype=torch.float64, device=net.device) for _ in range(4)]
    for a in range(0, N, chunk):
        b = min(N, a + chunk)
        f = net.predict_fields(re[a:b].contiguous(), u[a:b].contiguous(), H, W)
        for k in range(4):
            out[k][a:b].copy_(f[k])
    return out


def warm_start_batch(net, batch, re, u, cold_fields, check_steps=100, fallback_tol=1e-2, chunk=16):
    """Initialises every instance of `batch` (equal H x W cavities, instance order of
    re and u) at equilibrium with the network's predicted fields, advances check_steps
    steps and re-initialises at its cold state (cold_fields(i) -> (rho, ux, uy, phi))
    every instance whose velocity or scalar residual over those steps exceeds
    fallback_tol or that holds non-finite values.  Returns the fallback mask (numpy bool).
    The lattice Boltzmann run decides convergence: the prediction is only an initial state."""
    p0 = batch.problems[0]
    H, W = p0.ny, p0.nx
    if any(p.nx != W or p.ny != H for p in batch.problems):
        raise ValueError("warm_start_batch needs instances of one size")
    if check_steps % 2:
        raise ValueError("check_steps must be even")
    fields = predict_batch_fields(net, re, u, H, W, chunk)
    batch.init_device(*fields)
    del fields
    batch.reduce(raise_nonfinite=False)
    s = batch.step_reduce(check_steps, raise_nonfinite=False)
    ru, rp = s["res_u"], s["res_phi"]
    bad = (s["nonfinite"] > 0) | ~np.isfinite(ru) | ~np.isfinite(rp) | (ru > fallback_tol) | (rp > fallback_tol)
    for i in np.nonzero(bad)[0]:
        batch.init_instance(int(i), *cold_fields(int(i)))
    return bad


def train(net, re, u, targets, H, W, iters, batch_size=8, lr=1e-3, lr_min=1e-5, seed=0, log=None, log_every=100):
    """Adam on the weighted MSE with a cosine learning-rate schedule, on minibatches
    drawn without replacement (reshuffled every pass) from the N samples
    (re, u: float32 device [N]; targets: float32 device [N * H * W * 4])."""
    N = re.numel()
    tv = targets.view(N, H * W * 4)
    gen = torch.Generator().manual_seed(seed)
    order, pos = torch.randperm(N, generator=gen), 0
    hist = []
    for it in range(iters):
        if pos + batch_size > N:
            order, pos = torch.randperm(N, generator=gen), 0
        idx = order[pos:pos + batch_size].to(net.device)
        pos += batch_size
        lr_t = lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * it / max(1, iters)))
        loss = net.train_step(re[idx].contiguous(), u[idx].contiguous(), tv[idx].reshape(-1).contiguous(), H, W, lr_t)
        if log is not None and (it % log_every == 0 or it == iters - 1):
            v = loss.item()
            hist.append((it, v))
            log(it, v, lr_t)
    return hist


def evaluate_loss(net, re, u, targets, H, W, chunk=16):
    """Mean squared error per pixel (summed over the four channels) over N samples."""
    N = re.numel()
    tv = targets.view(N, H * W * 4)
    tot = 0.0
    for a in range(0, N, chunk):
        b = min(N, a + chunk)
        net.inputs(re[a:b].contiguous(), u[a:b].contiguous(), H, W)
        net.forward(b - a, H, W)
        tot += net.loss_and_grad(tv[a:b].reshape(-1).contiguous(), b - a, H, W).item() * (b - a)
    return tot / N


def save_weights(net, path, **meta):
    np.savez_compressed(path, w=net.w.detach().cpu().numpy(), base=np.int32(net.base), levels=np.int32(net.levels),
                        cin=np.int32(CIN), **{k: np.asarray(v) for k, v in meta.items()})


def load_weights(path, device="cuda"):
    with np.load(path, allow_pickle=False) as z:
        if "cin" not in z.files or int(z["cin"]) != CIN:
            raise ValueError(f"{path}: weights for a different input encoding (expected {CIN} input channels)")
        net = UNet(base=int(z["base"]), levels=int(z["levels"]), device=device)
        net.load_state_dict({"w": z["w"], "base": int(z["base"]), "levels": int(z["levels"])})
        meta = {k: z[k] for k in z.files if k not in ("w", "base", "levels", "cin")}
    return net, meta


def make_targets(rho, ux, uy, phi, u):
    """Normalised training targets [B*H*W*4] (float32) from FP64 fields [B, H, W]."""
    B = u.numel()
    HW = rho[0].numel()
    t = torch.empty(B * HW * 4, dtype=torch.float32, device=rho.device)
    L.check(L.lib().ddf_nn_cavity_targets(_p(rho), _p(ux), _p(uy), _p(phi), _p(u), B, HW, _p(t),
                                          C.c_void_p(torch.cuda.current_stream().cuda_stream)))
    return t
