"""FP64 CPU oracle for the DDF lattice Boltzmann method with local vorticity.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(the HIP library and its binding) never imports, links or calls it, and this
package imports nothing from the product package.

It wraps ``ddf_oracle.c`` (plain C, FP64, two-array pull streaming; see that
file's header for the paper passages each function follows) through ctypes.
Populations are numpy arrays of shape (9, ny, nx), direction-major, in the
paper's D2Q9 order (Sec. 2, eq. particlevelocities1/2).

Parity notes: every function here is pinned by ``tests/test_oracle_*.py``
against closed forms, invariants and the matrices printed in App. B.  The
scalar-model variants of App. C and App. D are pinned against each other and
against the closed-form flows.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ddf_oracle.c")
_LIB = os.path.join(_HERE, "libddf_oracle.so")

NQ = 9
OUTPUTS = ("rho", "ux", "uy", "phi", "Sxx", "Syy", "Sxy", "wz",
           "dxuy", "dyux", "dxphi", "dyphi", "Q", "R", "Lx", "Ly")

SCALAR_MODELS = {"mrt": 0, "srt": 1, "cascaded": 2, "central": 3}
FORCE_KINDS = {"none": 0, "uniform": 1, "fourroll": 2, "pulsatile": 3}


def build_command():
    return ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
            "-o", _LIB, _SRC, "-lm"]


def build(force: bool = True) -> str:
    """Compile the oracle shared library in place (plain gcc, no HIP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.check_call(build_command())
    return _LIB


class _Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int), ("ny", C.c_int),
        ("periodic_x", C.c_int), ("periodic_y", C.c_int),
        ("lam_f", C.c_double * NQ), ("lam_g", C.c_double * NQ),
        ("beta1", C.c_double), ("beta2", C.c_double),
        ("cs2", C.c_double), ("cs2phi", C.c_double),
        ("wall_ux", C.c_double * 4), ("wall_uy", C.c_double * 4),
        ("wall_phi", C.c_double * 4),
        ("force_kind", C.c_int),
        ("force", C.c_double * 2),
        ("force_k", C.c_double),
        ("force_omega", C.c_double),
        ("scalar_model", C.c_int),
        ("phi_min", C.c_double),
        ("nthreads", C.c_int),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        P = C.POINTER(_Params)
        L.orc_sizeof_params.restype = C.c_int
        L.orc_matrices.argtypes = [dp, dp, dp, dp]
        L.orc_meq_fluid.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, dp]
        L.orc_neq_scalar.argtypes = [C.c_double] * 6 + [dp]
        L.orc_source_moments.argtypes = [C.c_double] * 4 + [dp]
        L.orc_collide_node.argtypes = [P, dp, dp, C.c_double, C.c_double, dp, dp]
        L.orc_init.argtypes = [P, dp, dp, dp, dp, dp, dp]
        L.orc_step.argtypes = [P, dp, dp, C.c_long, C.c_long]
        L.orc_step.restype = C.c_int
        L.orc_extract_node.argtypes = [P, dp, dp, C.c_double, C.c_double, dp]
        L.orc_extract.argtypes = [P, dp, dp, C.c_long, dp]
        L.orc_force.argtypes = [P, C.c_int, C.c_int, C.c_double, dp]
        if L.orc_sizeof_params() != C.sizeof(_Params):
            raise RuntimeError("oracle parameter struct layout mismatch")
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


@dataclass
class Oracle:
    """Parameters of one lattice, converted from a problem description.

    ``problem`` is any object with the attributes of ``workloads.Problem``
    (grid, relaxation times, beta, walls, force).  The relaxation diagonals follow
    the paper's parameterisation: omega4 = omega5 = 1/tau (Sec. 5), bulk omega3 and
    the higher fluid rates from the problem, omega1^phi = omega2^phi = 1/tau_phi
    and the higher scalar rates from the problem.
    """

    problem: object
    nthreads: int = 0

    def __post_init__(self):
        pr = self.problem
        p = _Params()
        p.nx, p.ny = int(pr.nx), int(pr.ny)
        p.periodic_x, p.periodic_y = int(bool(pr.periodic_x)), int(bool(pr.periodic_y))
        w = 1.0 / pr.tau
        lam_f = [0.0, 0.0, 0.0, pr.omega3, w, w] + list(pr.omega_hi)
        wp = 1.0 / pr.tau_phi
        lam_g = [0.0, wp, wp] + list(pr.omega_phi_hi)
        if pr.scalar_model == "srt":
            lam_g = [0.0] + [wp] * 8
        p.lam_f[:] = lam_f
        p.lam_g[:] = lam_g
        p.beta1, p.beta2 = pr.beta1, pr.beta2
        p.cs2, p.cs2phi = pr.cs2, pr.cs2phi
        p.wall_ux[:] = [u[0] for u in pr.wall_u]
        p.wall_uy[:] = [u[1] for u in pr.wall_u]
        p.wall_phi[:] = [float("nan") if v is None else float(v) for v in pr.wall_phi]
        p.force_kind = FORCE_KINDS[pr.force_kind]
        p.force[:] = list(pr.force)
        p.force_k = pr.force_k
        p.force_omega = pr.force_omega
        p.scalar_model = SCALAR_MODELS[pr.scalar_model]
        p.phi_min = pr.phi_min
        p.nthreads = int(self.nthreads)
        self._p = p

    @property
    def params(self):
        return self._p

    @property
    def lam_f(self):
        return np.array(self._p.lam_f[:])

    @property
    def lam_g(self):
        return np.array(self._p.lam_g[:])

    def init(self, rho, ux, uy, phi):
        pr = self.problem
        shape = (pr.ny, pr.nx)
        args = [np.ascontiguousarray(np.broadcast_to(np.asarray(a, np.float64), shape)) for a in (rho, ux, uy, phi)]
        f = np.empty((NQ,) + shape)
        g = np.empty((NQ,) + shape)
        lib().orc_init(C.byref(self._p), *[_dp(a) for a in args], _dp(f), _dp(g))
        return f, g

    def step(self, f, g, nsteps, t0=0):
        rc = lib().orc_step(C.byref(self._p), _dp(f), _dp(g), int(nsteps), int(t0))
        if rc != 0:
            raise MemoryError("oracle step allocation failed")

    def extract(self, f, g, t=0):
        pr = self.problem
        out = np.empty((len(OUTPUTS), pr.ny, pr.nx))
        lib().orc_extract(C.byref(self._p), _dp(f), _dp(g), int(t), _dp(out))
        return {k: out[i] for i, k in enumerate(OUTPUTS)}

    def extract_node(self, f, g, F=(0.0, 0.0)):
        o = np.empty(len(OUTPUTS))
        f = np.ascontiguousarray(f, np.float64)
        g = np.ascontiguousarray(g, np.float64)
        lib().orc_extract_node(C.byref(self._p), _dp(f), _dp(g), float(F[0]), float(F[1]), _dp(o))
        return {k: o[i] for i, k in enumerate(OUTPUTS)}

    def collide_node(self, f, g, F=(0.0, 0.0)):
        f = np.ascontiguousarray(f, np.float64)
        g = np.ascontiguousarray(g, np.float64)
        fs = np.empty(NQ)
        gs = np.empty(NQ)
        lib().orc_collide_node(C.byref(self._p), _dp(f), _dp(g), float(F[0]), float(F[1]), _dp(fs), _dp(gs))
        return fs, gs

    def force(self, i, j, t=0.0):
        F = np.empty(2)
        lib().orc_force(C.byref(self._p), int(i), int(j), float(t), _dp(F))
        return F

    def run(self, fields, nsteps, t0=0):
        """Initialise from (rho, ux, uy, phi), advance nsteps, return (f, g, outputs)."""
        f, g = self.init(*fields)
        self.step(f, g, nsteps, t0)
        return f, g, self.extract(f, g, t0 + nsteps)


def matrices():
    """T, T^-1, P, P^-1 as built by the oracle from the basis definitions."""
    mats = [np.empty((NQ, NQ)) for _ in range(4)]
    lib().orc_matrices(*[_dp(m) for m in mats])
    return tuple(mats)


def meq_fluid(rho, ux, uy, cs2=1.0 / 3.0):
    out = np.empty(NQ)
    lib().orc_meq_fluid(rho, ux, uy, cs2, _dp(out))
    return out


def neq_scalar(phi, ux, uy, cs2phi=1.0 / 3.0, beta1=1.0, beta2=0.9):
    out = np.empty(NQ)
    lib().orc_neq_scalar(phi, ux, uy, cs2phi, beta1, beta2, _dp(out))
    return out


def source_moments(Fx, Fy, ux, uy):
    out = np.empty(NQ)
    lib().orc_source_moments(Fx, Fy, ux, uy, _dp(out))
    return out


def fd_curl(ux, uy, periodic=True):
    """Second-order central finite-difference vorticity (dx = 1), used only as an
    independent cross-check of the local extraction on smooth periodic fields."""
    if not periodic:
        raise NotImplementedError
    dvdx = (np.roll(uy, -1, axis=1) - np.roll(uy, 1, axis=1)) / 2.0
    dudy = (np.roll(ux, -1, axis=0) - np.roll(ux, 1, axis=0)) / 2.0
    return dvdx - dudy


def rel_l2(a, b):
    return float(math.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))
