"""The HBM reference kernels (include/ddf_probe.h) move exactly the bytes they claim:
the copy reproduces its source bit for bit, the write pass zeroes its destination and
the read pass leaves every buffer untouched."""
import ctypes as C

import pytest
import torch

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
