"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module holds problem descriptions (grid, relaxation times, walls, force) and
initial macroscopic fields (rho, u, phi) only.  It contains none of the lattice
Boltzmann arithmetic: no moments, equilibria, collision or streaming.  Both the
GPU library binding and the CPU oracle read these descriptions and convert them
with their own code.

Field arrays are float64, shape (ny, nx), indexed [y, x]; node (i, j) sits at
x = i, y = j in lattice units (dx = dt = 1, Sec. 5).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Optional, Sequence, Tuple

import numpy as np

CS2 = 1.0 / 3.0


@dataclass
class Problem:
    nx: int
    ny: int
    periodic_x: bool = True
    periodic_y: bool = True
    tau: float = 0.8                # omega4 = omega5 = 1/tau
    tau_phi: float = 0.7            # omega1^phi = omega2^phi = 1/tau_phi
    omega3: float = 1.0             # bulk rate (the paper leaves it unset; 1.0 is the default here)
    omega_hi: Tuple[float, float, float] = (1.0, 1.0, 1.0)                        # omega6..omega8
    omega_phi_hi: Tuple[float, ...] = (1.0, 1.0, 1.0, 1.0, 1.0, 1.0)              # omega3^phi..omega8^phi
    beta1: float = 1.0
    beta2: float = 0.9
    cs2: float = CS2
    cs2phi: float = CS2
    # walls, side order: left (x=-1/2), right (x=nx-1/2), bottom (y=-1/2), top (y=ny-1/2)
    wall_u: Sequence[Tuple[float, float]] = ((0.0, 0.0),) * 4
    wall_phi: Sequence[Optional[float]] = (None, None, None, None)   # None = zero-flux wall
    force_kind: str = "none"        # none | uniform | fourroll | pulsatile
    force: Tuple[float, float] = (0.0, 0.0)
    force_k: float = 0.0
    force_omega: float = 0.0
    scalar_model: str = "mrt"       # mrt | srt | cascaded | central
    phi_min: float = 1e-3
    # storage parameters of the GPU path (ignored by the oracle)
    storage: str = "f64"            # f64 | f32 | f16 | bf16
    rho0: float = 1.0
    phi0: float = 1.0
    layout: str = "auto"            # row layout of the population planes: auto | row | interleaved | packed

    def with_(self, **kw) -> "Problem":
        return replace(self, **kw)

    @property
    def nu(self) -> float:
        return self.cs2 * (self.tau - 0.5)

    @property
    def diffusivity(self) -> float:
        return self.cs2phi * (self.tau_phi - 0.5)


def grid(nx: int, ny: int):
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64), indexing="ij")
    return x, y


# --------------------------------------------------------------------------
# Taylor-Green vortex (64^2 periodic, FP64 workload)
# --------------------------------------------------------------------------

def taylor_green_problem(n: int = 64, tau: float = 0.8, tau_phi: float = 0.7, **kw) -> Problem:
    return Problem(nx=n, ny=n, tau=tau, tau_phi=tau_phi, **kw)


def taylor_green_fields(n: int, u0: float = 0.01, phi_amp: float = 0.1, phi_bg: float = 1.0,
                        uniform_phi: bool = False, x=None, y=None):
    """u = u0 sin kx cos ky, v = -u0 cos kx sin ky, k = 2 pi / n; rho = 1 + 3 p' with
    p' = (u0^2/4)(cos 2kx + cos 2ky); phi = phi_bg + phi_amp sin kx sin ky (or phi_bg)."""
    if x is None:
        x, y = grid(n, n)
    k = 2.0 * math.pi / n
    ux = u0 * np.sin(k * x) * np.cos(k * y)
    uy = -u0 * np.cos(k * x) * np.sin(k * y)
    p = (u0 * u0 / 4.0) * (np.cos(2 * k * x) + np.cos(2 * k * y))
    rho = 1.0 + p / CS2
    if uniform_phi:
        phi = np.full_like(x, phi_bg)
    else:
        phi = phi_bg + phi_amp * np.sin(k * x) * np.sin(k * y)
    return rho, ux, uy, phi


# --------------------------------------------------------------------------
# Channel flows (Poiseuille, Couette, Womersley)
# --------------------------------------------------------------------------

def channel_problem(nx: int, ny: int, tau: float, tau_phi: float = 0.57, force=(0.0, 0.0),
                    phi_bottom: Optional[float] = 1.0, phi_top: Optional[float] = 2.0,
                    u_top: float = 0.0, force_kind: str = "uniform", **kw) -> Problem:
    return Problem(nx=nx, ny=ny, periodic_x=True, periodic_y=False, tau=tau, tau_phi=tau_phi,
                   wall_u=((0.0, 0.0), (0.0, 0.0), (0.0, 0.0), (u_top, 0.0)),
                   wall_phi=(None, None, phi_bottom, phi_top),
                   force_kind=force_kind, force=tuple(force), **kw)


def rest_fields(nx: int, ny: int, rho: float = 1.0, phi: float = 1.0):
    z = np.zeros((ny, nx))
    return rho + z, z.copy(), z.copy(), phi + z


# --------------------------------------------------------------------------
# Four-rolls mill (Sec. 5.2)
# --------------------------------------------------------------------------

def fourroll_problem(n: int, nu_phys: float, u0: float, tau_phi: float = 0.57, **kw) -> Problem:
    """Periodic 2 pi x 2 pi domain on n^2 nodes, dx = dt = 2 pi / n.  The lattice
    viscosity is nu_phys * dt / dx^2 and the force amplitude 2 rho0 nu_lat u0 k^2."""
    k = 2.0 * math.pi / n
    nu_lat = nu_phys / k
    tau = 0.5 + nu_lat / CS2
    amp = 2.0 * 1.0 * nu_lat * u0 * k * k
    return Problem(nx=n, ny=n, tau=tau, tau_phi=tau_phi, force_kind="fourroll",
                   force=(amp, 0.0), force_k=k, **kw)


def fourroll_fields(n: int, u0: float, phi: float = 2.0, x=None, y=None):
    if x is None:
        x, y = grid(n, n)
    k = 2.0 * math.pi / n
    ux = u0 * np.sin(k * x) * np.sin(k * y)
    uy = u0 * np.cos(k * x) * np.cos(k * y)
    return np.ones_like(x), ux, uy, np.full_like(x, phi)


# --------------------------------------------------------------------------
# Lid-driven cavity (1024^2 FP32 workload and smaller instances)
# --------------------------------------------------------------------------

def cavity_problem(n: int, re: float, u_lid: float, phi_lid: float = 1.0, phi_walls: float = 0.0,
                   storage: str = "f32", **kw) -> Problem:
    nu = u_lid * n / re
    tau = 0.5 + nu / CS2
    return Problem(nx=n, ny=n, periodic_x=False, periodic_y=False, tau=tau, tau_phi=tau,
                   wall_u=((0.0, 0.0), (0.0, 0.0), (0.0, 0.0), (u_lid, 0.0)),
                   wall_phi=(phi_walls, phi_walls, phi_walls, phi_lid),
                   storage=storage, rho0=1.0, phi0=0.5, **kw)


def cavity_fields(n: int, phi_inside: float = 0.0):
    return rest_fields(n, n, 1.0, phi_inside)


# --------------------------------------------------------------------------
# Periodic decaying vortex field (8192^2 workload, and crops of it)
# --------------------------------------------------------------------------

@dataclass
class VortexField:
    """Seeded random streamfunction psi = sum a_k cos(2 pi k.x / L + theta_k) over
    4 <= |k| <= 16 (one mode per +-k pair), a_k ~ N(0,1)/|k|, theta_k ~ U[0, 2 pi),
    scaled so that max |u| = u_max; and a scalar phi = 1 + sum_j a_j
    exp(-d_per(x, c_j)^2 / (2 sigma^2)) with n_blobs Gaussian blobs, c_j ~ U[0, L)^2,
    a_j ~ U(0.1, 0.5).  Evaluated analytically at any node set."""

    L: int = 8192
    u_max: float = 0.02
    kmin: float = 4.0
    kmax: float = 16.0
    n_blobs: int = 1024
    sigma: float = 32.0
    seed_modes: int = 1908
    seed_blobs: int = 6742
    scale: float = field(default=0.0, init=False)

    def __post_init__(self):
        rng = np.random.default_rng(self.seed_modes)
        ks = []
        K = int(self.kmax)
        for kx in range(0, K + 1):
            for ky in range(-K, K + 1):
                if kx == 0 and ky <= 0:
                    continue  # one mode per +-k pair
                r = math.hypot(kx, ky)
                if self.kmin <= r <= self.kmax:
                    ks.append((kx, ky))
        self.modes = np.array(ks, dtype=np.float64)
        nm = len(ks)
        self.amp = rng.standard_normal(nm) / np.hypot(self.modes[:, 0], self.modes[:, 1])
        self.theta = rng.uniform(0.0, 2.0 * math.pi, nm)
        rb = np.random.default_rng(self.seed_blobs)
        self.centers = rb.uniform(0.0, self.L, (self.n_blobs, 2))
        self.blob_amp = rb.uniform(0.1, 0.5, self.n_blobs)
        # max |u| of the unscaled field, taken on a tensor grid of stride L/1024
        # (the shortest wavelength is L/16, so this resolves every extremum).
        self.scale = 1.0
        s = max(1, self.L // 1024)
        coords = np.arange(0, self.L, s, dtype=np.float64)
        _, ux, uy, _ = self.eval_grid(coords, coords, with_scalar=False)
        self.scale = self.u_max / float(np.max(np.hypot(ux, uy)))

    def eval_grid(self, xs, ys, with_scalar=True, device="cpu"):
        """Fields on the tensor grid xs (columns) x ys (rows), float64 numpy arrays
        [len(ys), len(xs)], by separable matrix products (torch, any device)."""
        import torch
        L = self.L
        w = 2.0 * math.pi / L
        X = torch.as_tensor(np.asarray(xs, np.float64), device=device)
        Y = torch.as_tensor(np.asarray(ys, np.float64), device=device)
        kx = torch.tensor(self.modes[:, 0], device=device, dtype=torch.float64)
        ky = torch.tensor(self.modes[:, 1], device=device, dtype=torch.float64)
        a = torch.tensor(self.amp, device=device, dtype=torch.float64) * self.scale
        th = torch.tensor(self.theta, device=device, dtype=torch.float64)
        # psi = a cos(w kx x + w ky y + th); u = d psi/dy, v = -d psi/dx, and
        # sin(P + R) = sin P cos R + cos P sin R with P = w kx x + th, R = w ky y
        Pm = w * X[:, None] * kx[None, :] + th[None, :]
        Rm = w * Y[:, None] * ky[None, :]
        sP, cP, sR, cR = torch.sin(Pm), torch.cos(Pm), torch.sin(Rm), torch.cos(Rm)
        cu = -a * w * ky
        cv = a * w * kx
        ux = (cR * cu) @ sP.T + (sR * cu) @ cP.T
        uy = (cR * cv) @ sP.T + (sR * cv) @ cP.T
        phi = None
        if with_scalar:
            cxy = torch.tensor(self.centers, device=device, dtype=torch.float64)
            amp = torch.tensor(self.blob_amp, device=device, dtype=torch.float64)
            dx = (X[:, None] - cxy[None, :, 0]).abs()
            dx = torch.minimum(dx, L - dx)
            dy = (Y[:, None] - cxy[None, :, 1]).abs()
            dy = torch.minimum(dy, L - dy)
            gx = torch.exp(-dx * dx / (2.0 * self.sigma ** 2))
            gy = torch.exp(-dy * dy / (2.0 * self.sigma ** 2))
            phi = 1.0 + (gy * amp) @ gx.T
        rho = torch.ones_like(ux)
        if device == "cpu":
            return (rho.numpy(), ux.numpy(), uy.numpy(), None if phi is None else phi.numpy())
        return rho, ux, uy, phi

    def fields(self, x0=0, y0=0, nx=None, ny=None):
        """Fields on the window [x0, x0+nx) x [y0, y0+ny), coordinates taken modulo L."""
        nx = self.L if nx is None else nx
        ny = self.L if ny is None else ny
        xs = np.arange(x0, x0 + nx) % self.L
        ys = np.arange(y0, y0 + ny) % self.L
        return self.eval_grid(xs, ys)


def vortex_problem(L: int = 8192, storage: str = "f32", **kw) -> Problem:
    return Problem(nx=L, ny=L, tau=0.8, tau_phi=0.7, storage=storage, rho0=1.0, phi0=1.0, **kw)


# --------------------------------------------------------------------------
# Batched cavities and channels (256 instances of uneven size)
# --------------------------------------------------------------------------

@dataclass
class Instance:
    kind: str       # cavity | channel
    nx: int
    ny: int
    re: float
    u: float
    problem: Problem


def batch_instances(count: int = 256, seed0: int = 4096, side_lo: int = 64, side_hi: int = 512,
                    storage: str = "f32"):
    """Instance i uses seed seed0 + i: kind ~ Bernoulli(1/2) cavity/channel, sides ~ U{lo..hi}
    (square cavities; channels of height H and length W), Re log-uniform in [100, 5000],
    U ~ U(0.05, 0.1), tau = 1/2 + 3 U L / Re, tau_phi = tau.  Channels are periodic in x,
    with half-way walls at bottom and top and the body force 8 rho nu U / H^2 that gives
    centre-line speed U; phi walls 1 (bottom) and 0 (top).  Cavities follow the 1024^2
    cavity workload (lid phi = 1, other walls phi = 0)."""
    out = []
    for i in range(count):
        r = np.random.default_rng(seed0 + i)
        kind = "cavity" if r.random() < 0.5 else "channel"
        re = float(math.exp(r.uniform(math.log(100.0), math.log(5000.0))))
        u = float(r.uniform(0.05, 0.1))
        if kind == "cavity":
            n = int(r.integers(side_lo, side_hi + 1))
            pr = cavity_problem(n, re, u, storage=storage)
            out.append(Instance(kind, n, n, re, u, pr))
        else:
            H = int(r.integers(side_lo, side_hi + 1))
            W = int(r.integers(side_lo, side_hi + 1))
            nu = u * H / re
            tau = 0.5 + nu / CS2
            F = 8.0 * 1.0 * nu * u / (H * H)
            pr = Problem(nx=W, ny=H, periodic_x=True, periodic_y=False, tau=tau, tau_phi=tau,
                         wall_u=((0.0, 0.0),) * 4, wall_phi=(None, None, 1.0, 0.0),
                         force_kind="uniform", force=(F, 0.0), storage=storage, rho0=1.0, phi0=0.5)
            out.append(Instance(kind, W, H, re, u, pr))
    return out


# --------------------------------------------------------------------------
# Cavity family of the surrogate study
# --------------------------------------------------------------------------

SURROGATE_TRAIN_SEED0 = 0
SURROGATE_HELDOUT_SEED0 = 100_000


def surrogate_cases(count: int, seed0: int = SURROGATE_TRAIN_SEED0):
    """(Re, U) of cavity i from seed seed0 + i: Re log-uniform in [100, 5000],
    lid speed U ~ U(0.05, 0.1).  Training uses seeds 0.., held-out evaluation
    seeds 100000.."""
    out = []
    for i in range(count):
        r = np.random.default_rng(seed0 + i)
        re = float(math.exp(r.uniform(math.log(100.0), math.log(5000.0))))
        u = float(r.uniform(0.05, 0.1))
        out.append((re, u))
    return out
