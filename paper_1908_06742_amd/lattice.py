"""Python face of libddf: one coupled fluid + scalar D2Q9 lattice on one GPU.

Argument marshalling only: torch allocates the device buffers and supplies the
stream; every step of the method runs in the HIP kernels behind the C ABI.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib as L

_TORCH_STORAGE = {L.DDF_F64: torch.float64, L.DDF_F32: torch.float32,
                  L.DDF_F16: torch.float16, L.DDF_BF16: torch.bfloat16,
                  L.DDF_BF16_SR: torch.bfloat16}


def _stream_ptr(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor):
    return C.c_void_p(t.data_ptr())


_OUT_DTYPES = {torch.float64: 0, torch.float32: 1}


def _same_device(a: torch.device, b: torch.device) -> bool:
    if a.type != b.type:
        return False
    if a.type != "cuda" or a.index == b.index:
        return True
    cur = torch.cuda.current_device()
    return (a.index if a.index is not None else cur) == (b.index if b.index is not None else cur)


def out_dtype_code(dtype) -> int:
    """Output type code of the extraction calls (0 = float64, 1 = float32)."""
    if dtype not in _OUT_DTYPES:
        raise ValueError(f"extraction writes float64 or float32 planes, not {dtype}")
    return _OUT_DTYPES[dtype]


def output_mask(names) -> int:
    mask = 0
    for n in names:
        if n not in L.OUTPUTS:
            raise ValueError(f"unknown output {n!r}; choose from {L.OUTPUTS}")
        mask |= 1 << L.OUTPUTS.index(n)
    return mask


def check_extract_out(out, mask, ny, nx, device) -> int:
    """The extraction kernels write plane k of `out` (k * ny * nx elements in) for every
    bit k of mask: `out` must be a contiguous float32/float64 tensor on the lattice's
    device holding at least (highest bit + 1) planes.  Returns the dtype code."""
    if not torch.is_tensor(out):
        raise ValueError("out must be a torch tensor")
    code = out_dtype_code(out.dtype)
    if not _same_device(out.device, device):
        raise ValueError(f"out is on {out.device}, the lattice on {device}")
    if not out.is_contiguous():
        raise ValueError("out must be contiguous")
    need = mask.bit_length() * ny * nx
    if out.numel() < need:
        raise ValueError(f"out holds {out.numel()} elements; the selected outputs need {need} "
                         f"({mask.bit_length()} planes of {ny} x {nx})")
    return code


def check_field(t, n, what):
    """A dense field handed to the kernels, which read exactly n float64 elements."""
    if t.dtype != torch.float64 or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{what}: need a contiguous float64 tensor of {n} elements, got "
                         f"{tuple(t.shape)} {t.dtype}{'' if t.is_contiguous() else ' (not contiguous)'}")
    return t


def check_populations(t, ny, nx, what):
    """Logical populations, direction-major (9, ny, nx)."""
    if tuple(t.shape) != (9, ny, nx):
        raise ValueError(f"{what}: need shape (9, {ny}, {nx}), got {tuple(t.shape)}")
    return t


class Lattice:
    """A fluid lattice f and a scalar lattice g (caller-owned torch buffers).

    ``problem`` is a workloads.Problem (or any object with its attributes).
    """

    def __init__(self, problem, device="cuda", stream=None):
        lib = L.lib()
        self.problem = problem
        self.params = L.params_from_problem(problem)
        self.device = torch.device(device)
        self.stream = stream
        nbytes = lib.ddf_population_bytes(C.byref(self.params))
        wbytes = lib.ddf_workspace_bytes(C.byref(self.params))
        if nbytes == 0 or wbytes == 0:
            # validation failure: surface the library's message
            h = C.c_void_p()
            L.check(lib.ddf_create(C.byref(self.params), C.c_void_p(256), C.c_void_p(256), C.c_void_p(256), C.byref(h)))
        self.pop_f = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.pop_g = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.workspace = torch.empty(wbytes, dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        L.check(lib.ddf_create(C.byref(self.params), _ptr(self.pop_f), _ptr(self.pop_g), _ptr(self.workspace),
                               C.byref(h)))
        self._h = h
        self.nx, self.ny = int(problem.nx), int(problem.ny)
        self.pitch = int(lib.ddf_pitch(C.byref(self.params)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            try:
                L.lib().ddf_destroy(h)
            except TypeError:      # interpreter shutdown: module globals already cleared
                pass
            self._h = None

    # -- state -----------------------------------------------------------------
    def _field(self, a):
        t = torch.as_tensor(a, dtype=torch.float64)
        try:
            t = torch.broadcast_to(t, (self.ny, self.nx))
        except RuntimeError as e:
            raise ValueError(f"field of shape {tuple(t.shape)} does not broadcast to ({self.ny}, {self.nx})") from e
        return check_field(t.to(self.device).contiguous(), self.ny * self.nx, "field")

    def init(self, rho, ux, uy, phi):
        fields = [self._field(a) for a in (rho, ux, uy, phi)]
        L.check(L.lib().ddf_init_equilibrium(self._h, *[_ptr(t) for t in fields], _stream_ptr(self.stream)))
        self._keep = fields  # alive until the stream has consumed them
        return self

    def set_tile_width(self, bx_max):
        """Tile width of this lattice's kernels (64, 128, 256 or 512); results do not change."""
        L.check(L.lib().ddf_set_tile_width(self._h, int(bx_max)))
        return self

    @property
    def layout(self):
        """Row layout of the population planes ("row", "interleaved" or "packed"), chosen at creation."""
        return L.LAYOUT_NAMES[int(L.lib().ddf_get_layout(self._h))]

    @property
    def tile_width(self):
        return int(L.lib().ddf_get_tile_width(self._h))

    def set_address_width(self, bits):
        """Lane-offset width of the step kernels (32 where planes are below 4 GiB, or 64);
        results do not change."""
        L.check(L.lib().ddf_set_address_width(self._h, int(bits)))
        return self

    @property
    def address_width(self):
        return int(L.lib().ddf_get_address_width(self._h))

    def set_workgroups_per_cu(self, even, odd):
        """Resident step workgroups per CU for even and odd steps (0 = no limit, 1, 2 or 3);
        results do not change."""
        L.check(L.lib().ddf_set_workgroups_per_cu(self._h, int(even), int(odd)))
        return self

    @property
    def workgroups_per_cu(self):
        e, o = C.c_int32(), C.c_int32()
        L.check(L.lib().ddf_get_workgroups_per_cu(self._h, C.byref(e), C.byref(o)))
        return int(e.value), int(o.value)

    def pattern_probe(self, parity, wg_per_cu=0):
        """The step's memory accesses of one parity without its collision (a reference
        for the step's bandwidth): swaps opposite directions in each
        node's slot set and flips their signs, so two calls of one parity restore the
        populations."""
        L.check(L.lib().ddf_pattern_probe(self._h, int(parity), int(wg_per_cu), _stream_ptr(self.stream)))
        return self

    def set_graph(self, steps_per_graph):
        """Steps per captured hipGraph replay (even; 0 = eager launches)."""
        L.check(L.lib().ddf_set_graph(self._h, int(steps_per_graph)))
        return self

    def step(self, nsteps=1):
        L.check(L.lib().ddf_step(self._h, int(nsteps), _stream_ptr(self.stream)))
        return self

    @property
    def step_count(self):
        return int(L.lib().ddf_step_count(self._h))

    def extract(self, names=None, dtype=torch.float64, out=None):
        """Local kinematics of the current state: dict name -> (ny, nx) tensor."""
        names = list(L.OUTPUTS) if names is None else list(names)
        mask = output_mask(names)
        if out is None:
            out_dtype_code(dtype)
            out = torch.empty((len(L.OUTPUTS), self.ny, self.nx), dtype=dtype, device=self.device)
        od = check_extract_out(out, mask, self.ny, self.nx, self.device)
        L.check(L.lib().ddf_extract(self._h, _ptr(out), mask, od, _stream_ptr(self.stream)))
        flat, plane = out.view(-1), self.ny * self.nx
        return {n: flat[L.OUTPUTS.index(n) * plane:(L.OUTPUTS.index(n) + 1) * plane].view(self.ny, self.nx)
                for n in names}

    def reduce(self, raise_nonfinite=True):
        buf = (C.c_double * len(L.STATS))()
        rc = L.lib().ddf_reduce(self._h, buf, _stream_ptr(self.stream))
        stats = {k: buf[i] for i, k in enumerate(L.STATS)}
        if rc == L.DDF_ERR_NONFINITE and not raise_nonfinite:
            return stats
        L.check(rc)
        return stats

    def get_populations(self, raw=False):
        """(f, g) as (9, ny, nx): absolute float64 values, or the raw stored offsets."""
        dt = _TORCH_STORAGE[self.params.storage] if raw else torch.float64
        f = torch.empty((9, self.ny, self.nx), dtype=dt, device=self.device)
        g = torch.empty_like(f)
        L.check(L.lib().ddf_get_populations(self._h, _ptr(f), _ptr(g), 1 if raw else 0, _stream_ptr(self.stream)))
        return f, g

    def set_populations(self, f, g, step=0, raw=False):
        dt = _TORCH_STORAGE[self.params.storage] if raw else torch.float64
        f = check_populations(torch.as_tensor(f), self.ny, self.nx, "f").to(self.device, dt).contiguous()
        g = check_populations(torch.as_tensor(g), self.ny, self.nx, "g").to(self.device, dt).contiguous()
        L.check(L.lib().ddf_set_populations(self._h, _ptr(f), _ptr(g), 1 if raw else 0, int(step),
                                            _stream_ptr(self.stream)))
        self._keep = (f, g)
        return self
