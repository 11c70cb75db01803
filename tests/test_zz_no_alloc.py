"""ddf_nn_mse_static, the allocation-free variant of ddf_nn_mse (its partial sums live in
a fixed device array of the library), against ddf_nn_mse with a caller workspace and
against the FP64 reference: two calls in a row, the second smaller, so the second reads
an array that still holds the first call's partials."""
import ctypes as C

import numpy as np
import pytest
import torch

from oracle import unet as U
from paper_1908_06742_amd import _lib as L

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _p(t):
    return C.c_void_p(t.data_ptr())


def _inputs(npix, cs, seed):
    g = torch.Generator().manual_seed(seed)
    out = (torch.randn((npix, cs), generator=g) * 0.5).to(torch.bfloat16).to(DEV).contiguous()
    tgt = (torch.randn((npix, 4), generator=g) * 0.5).to(DEV).contiguous()
    return out, tgt


def _mse(out, tgt, npix, cs, w, static):
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    dout = torch.full_like(out, float("nan"))
    loss = torch.full((1,), float("nan"), dtype=torch.float64, device=DEV)
    wts = (C.c_float * 4)(*w)
    if static:
        L.check(L.lib().ddf_nn_mse_static(_p(out), cs, _p(tgt), npix, wts, _p(dout), _p(loss), s))
    else:
        ws = torch.empty(L.lib().ddf_nn_mse_workspace_bytes(npix), dtype=torch.uint8, device=DEV)
        L.check(L.lib().ddf_nn_mse(_p(out), cs, _p(tgt), npix, wts, _p(dout), _p(loss), _p(ws), s))
        torch.cuda.synchronize()
    torch.cuda.synchronize()
    return loss.item(), dout


def test_static_mse_equals_the_workspace_variant_on_two_calls_in_a_row():
    w = (1.0, 0.5, 2.0, 1.5)
    cap = int(L.lib().ddf_nn_mse_static_max_pixels())
    assert cap == 2_096_896
    # a large ragged call, then a small one over the array the first call filled
    for npix, cs, seed in ((cap - 77, 32, 1), (1000, 8, 2)):
        print(f"case: mse_static npix={npix} channel stride {cs}", flush=True)
        out, tgt = _inputs(npix, cs, seed)
        la, da = _mse(out, tgt, npix, cs, w, static=False)
        lb, db = _mse(out, tgt, npix, cs, w, static=True)
        assert la == lb, (npix, la, lb)
        assert torch.equal(da.view(torch.int16), db.view(torch.int16))
        # and both against the FP64 reference on the same BF16 inputs (the kernel forms
        # the differences in FP32: relative rounding about 1e-7)
        o = out[:, :4].double().cpu().numpy().reshape(1, 1, npix, 4)
        t = tgt.double().cpu().numpy().reshape(1, 1, npix, 4)
        rl, rg = U.mse(o, t, np.array(w))
        assert abs(lb - rl) <= 1e-6 * rl
        g = db[:, :4].double().cpu().numpy()
        assert np.max(np.abs(g - rg.reshape(npix, 4))) <= 2.0 ** -8 * np.max(np.abs(rg))
        assert torch.all(db[:, 4:] == 0)


def test_static_mse_refuses_more_pixels_than_its_array_holds():
    cap = int(L.lib().ddf_nn_mse_static_max_pixels())
    out, tgt = _inputs(16, 8, 3)
    wts = (C.c_float * 4)(1.0, 1.0, 1.0, 1.0)
    loss = torch.zeros(1, dtype=torch.float64, device=DEV)
    rc = L.lib().ddf_nn_mse_static(_p(out), 8, _p(tgt), cap + 1, wts, _p(out), _p(loss), None)
    assert rc == L.DDF_ERR_ARG and "exceeds" in L.lib().ddf_last_error().decode()
