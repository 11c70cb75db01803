"""Python face of the libddf batch API: many independent lattices stepped together.

Argument marshalling only; the stepping, reductions and extraction run in HIP.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L
from .lattice import _TORCH_STORAGE, _ptr, _stream_ptr, check_field, out_dtype_code, output_mask


class Batch:
    """``problems``: a list of workloads.Problem (one per instance)."""

    def __init__(self, problems, device="cuda", stream=None):
        lib = L.lib()
        self.problems = list(problems)
        self.n = len(self.problems)
        arr = (L.Params * self.n)(*[L.params_from_problem(p) for p in self.problems])
        self._params = arr
        self.device = torch.device(device)
        self.stream = stream
        nbytes = lib.ddf_batch_population_bytes(self.n, arr)
        wbytes = lib.ddf_batch_workspace_bytes(self.n, arr)
        if wbytes == 0:
            h = C.c_void_p()
            L.check(lib.ddf_batch_create(self.n, arr, C.c_void_p(256), C.c_void_p(256), C.c_void_p(256), C.byref(h)))
        self.pop_f = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.pop_g = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.workspace = torch.empty(wbytes, dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        L.check(lib.ddf_batch_create(self.n, arr, _ptr(self.pop_f), _ptr(self.pop_g), _ptr(self.workspace), C.byref(h)))
        self._h = h
        self.field_offsets = []
        for i in range(self.n):
            po, fo = C.c_int64(), C.c_int64()
            L.check(lib.ddf_batch_offsets(h, i, C.byref(po), C.byref(fo)))
            self.field_offsets.append(int(fo.value))
        self.total_nodes = sum(int(p.nx) * int(p.ny) for p in self.problems)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            try:
                L.lib().ddf_batch_destroy(h)
            except TypeError:      # interpreter shutdown: module globals already cleared
                pass
            self._h = None

    def init(self, fields):
        """fields: list of (rho, ux, uy, phi) per instance (arrays of shape (ny, nx))."""
        cat = []
        for k in range(4):
            parts = [torch.as_tensor(np.array(np.broadcast_to(np.asarray(f[k], np.float64), (p.ny, p.nx))))
                     .reshape(-1)
                     for f, p in zip(fields, self.problems)]
            cat.append(torch.cat(parts).to(self.device).contiguous())
        L.check(L.lib().ddf_batch_init_equilibrium(self._h, *[_ptr(t) for t in cat], _stream_ptr(self.stream)))
        self._keep = cat
        return self

    def init_device(self, rho, ux, uy, phi):
        """Initialise from concatenated FP64 device tensors (instance order, [ny][nx] each)."""
        fields = [check_field(t.to(self.device, torch.float64).contiguous().reshape(-1), self.total_nodes, nm)
                  for t, nm in zip((rho, ux, uy, phi), ("rho", "ux", "uy", "phi"))]
        L.check(L.lib().ddf_batch_init_equilibrium(self._h, *[_ptr(t) for t in fields], _stream_ptr(self.stream)))
        self._keep = fields
        return self

    def init_instance(self, i, rho, ux, uy, phi):
        p = self.problems[i]

        def dev(a, nm):
            if not torch.is_tensor(a):
                a = torch.as_tensor(np.array(np.broadcast_to(np.asarray(a, np.float64), (p.ny, p.nx))))
            return check_field(a.to(self.device, torch.float64).contiguous(), p.ny * p.nx, nm)

        fields = [dev(a, nm) for a, nm in zip((rho, ux, uy, phi), ("rho", "ux", "uy", "phi"))]
        L.check(L.lib().ddf_batch_init_instance(self._h, int(i), *[_ptr(t) for t in fields], _stream_ptr(self.stream)))
        self._keep_i = fields
        return self

    def set_active(self, active):
        a = (C.c_uint8 * self.n)(*[1 if x else 0 for x in active])
        L.check(L.lib().ddf_batch_set_active(self._h, a))

    def autotune(self, steps_per_trial=20):
        bx, bpc, ms = C.c_int32(), C.c_int32(), C.c_float()
        L.check(L.lib().ddf_batch_autotune(self._h, int(steps_per_trial), C.byref(bx), C.byref(bpc), C.byref(ms),
                                           _stream_ptr(self.stream)))
        return {"bx_max": bx.value, "blocks_per_cu": bpc.value, "nontemporal": list(self.nontemporal),
                "ms_per_step": ms.value}

    def set_nontemporal(self, even, odd):
        """Non-temporal loads and stores in the even / odd step kernel; results do not change."""
        L.check(L.lib().ddf_batch_set_nontemporal(self._h, int(bool(even)), int(bool(odd))))

    @property
    def nontemporal(self):
        e, o = C.c_int32(), C.c_int32()
        L.check(L.lib().ddf_batch_get_nontemporal(self._h, C.byref(e), C.byref(o)))
        return int(e.value), int(o.value)

    def set_tiling(self, bx_max, blocks_per_cu):
        L.check(L.lib().ddf_batch_set_tiling(self._h, int(bx_max), int(blocks_per_cu)))

    def tiling(self):
        v = [C.c_int32() for _ in range(4)]
        L.check(L.lib().ddf_batch_get_tiling(self._h, *[C.byref(x) for x in v]))
        return dict(zip(("bx_max", "blocks_per_cu", "ntiles", "grid"), [x.value for x in v]))

    def pattern_probe(self, parity):
        """The batch step's memory accesses of one parity without its collision (a
        reference for its bandwidth): swaps opposite directions in each node's slot set
        and flips their signs, so two calls of one parity restore the populations."""
        L.check(L.lib().ddf_batch_pattern_probe(self._h, int(parity), _stream_ptr(self.stream)))
        return self

    def set_graph(self, steps_per_graph):
        L.check(L.lib().ddf_batch_set_graph(self._h, int(steps_per_graph)))

    def step(self, nsteps=1):
        L.check(L.lib().ddf_batch_step(self._h, int(nsteps), _stream_ptr(self.stream)))
        return self

    @property
    def step_count(self):
        return int(L.lib().ddf_batch_step_count(self._h))

    def reduce(self, raise_nonfinite=False):
        """Per-instance statistics: dict name -> numpy array of length n."""
        buf = (C.c_double * (self.n * len(L.STATS)))()
        rc = L.lib().ddf_batch_reduce(self._h, buf, _stream_ptr(self.stream))
        return self._stats(buf, rc, raise_nonfinite)

    def step_reduce(self, nsteps, raise_nonfinite=False):
        """step(nsteps) then reduce(), with the reduction inside the last graph replay
        where the run ends on one."""
        buf = (C.c_double * (self.n * len(L.STATS)))()
        rc = L.lib().ddf_batch_step_reduce(self._h, int(nsteps), buf, _stream_ptr(self.stream))
        return self._stats(buf, rc, raise_nonfinite)

    def _stats(self, buf, rc, raise_nonfinite):
        if rc != L.DDF_OK and not (rc == L.DDF_ERR_NONFINITE and not raise_nonfinite):
            L.check(rc)
        a = np.frombuffer(buf, dtype=np.float64).reshape(self.n, len(L.STATS)).copy()
        return {k: a[:, i] for i, k in enumerate(L.STATS)}

    def extract(self, i, names=None, dtype=torch.float64):
        p = self.problems[i]
        names = list(L.OUTPUTS) if names is None else list(names)
        mask = output_mask(names)
        od = out_dtype_code(dtype)
        out = torch.empty((len(L.OUTPUTS), p.ny, p.nx), dtype=dtype, device=self.device)
        L.check(L.lib().ddf_batch_extract(self._h, int(i), _ptr(out), mask, od, _stream_ptr(self.stream)))
        return {nm: out[L.OUTPUTS.index(nm)] for nm in names}

    def get_populations(self, i, raw=False):
        p = self.problems[i]
        dt = _TORCH_STORAGE[L.STORAGE[p.storage]] if raw else torch.float64
        f = torch.empty((9, p.ny, p.nx), dtype=dt, device=self.device)
        g = torch.empty_like(f)
        L.check(L.lib().ddf_batch_get_populations(self._h, int(i), _ptr(f), _ptr(g), 1 if raw else 0,
                                                  _stream_ptr(self.stream)))
        return f, g
