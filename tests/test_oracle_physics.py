"""Pins of the oracle's time stepping and extraction against closed-form flows.

Closed forms used (none of them computed by the oracle):
  - Taylor-Green decay of u, of omega and of a scalar aligned with the streamfunction;
  - plane Poiseuille flow omega_z = 2 U_max y / L^2 (Sec. 5.1);
  - plane Couette flow omega_z = -U / H and the linear Dirichlet scalar profile;
  - four-rolls mill omega_z = -2 u0 sin x cos y (Sec. 5.2) and second-order convergence (Sec. 5.2.1);
  - Womersley flow (Sec. 5.3), with the sign-corrected closed form;
  - exact conservation of mass and scalar, and finite-difference curl on smooth fields.
"""
import cmath
import math

import numpy as np
import pytest

import oracle
import workloads as W


def tg_closed_form(n, u0, nu, D, t, phi_amp=0.1, phi_bg=1.0):
    x, y = W.grid(n, n)
    k = 2.0 * math.pi / n
    eu = math.exp(-2.0 * nu * k * k * t)
    ep = math.exp(-2.0 * D * k * k * t)
    ux = u0 * np.sin(k * x) * np.cos(k * y) * eu
    uy = -u0 * np.cos(k * x) * np.sin(k * y) * eu
    wz = 2.0 * u0 * k * np.sin(k * x) * np.sin(k * y) * eu
    phi = phi_bg + phi_amp * np.sin(k * x) * np.sin(k * y) * ep
    dxdyphi = phi_amp * k * k * np.cos(k * x) * np.cos(k * y) * ep
    return ux, uy, wz, phi, dxdyphi


@pytest.fixture(scope="module")
def tg_runs(nthreads):
    """Taylor-Green, tau = 0.8, tau_phi = 0.7, u0 = 0.01 at 32^2 and 64^2 (1000 steps at 64^2,
    the same diffusive time at 32^2), literal sin sin scalar and the uniform-scalar twin."""
    runs = {}
    for n, steps in ((32, 250), (64, 1000)):
        pr = W.taylor_green_problem(n)
        o = oracle.Oracle(pr, nthreads=nthreads)
        for uniform in (False, True):
            f, g, out = o.run(W.taylor_green_fields(n, 0.01, uniform_phi=uniform), steps)
            runs[(n, uniform)] = (pr, steps, out, f, g)
    return runs


def test_taylor_green_velocity_and_scalar_decay(tg_runs):
    errs_u, errs_p = [], []
    for n in (32, 64):
        pr, t, out, _, _ = tg_runs[(n, False)]
        ux, uy, _, phi, _ = tg_closed_form(n, 0.01, pr.nu, pr.diffusivity, t)
        errs_u.append(oracle.rel_l2(out["ux"], ux))
        errs_p.append(oracle.rel_l2(out["phi"] - 1.0, phi - 1.0))
    assert errs_u[1] < 1.5e-3 and errs_p[1] < 2.5e-3
    # second order: the error drops by ~4 when the grid is refined at fixed diffusive time
    assert 3.5 < errs_u[0] / errs_u[1] < 4.5
    assert 3.0 < errs_p[0] / errs_p[1] < 5.0


def test_taylor_green_vorticity_uniform_scalar_second_order(tg_runs):
    e = []
    for n in (32, 64):
        pr, t, out, _, _ = tg_runs[(n, True)]
        _, _, wz, _, _ = tg_closed_form(n, 0.01, pr.nu, pr.diffusivity, t)
        e.append(oracle.rel_l2(out["wz"], wz))
    assert e[1] < 8e-3
    assert 3.5 < e[0] / e[1] < 4.5


def test_taylor_green_curved_scalar_shows_dropped_second_order_term(tg_runs):
    # The paper's relation for n5 stops at O(epsilon).  The O(epsilon^2) term of the
    # scalar moment system (App. A structure) adds
    #   -2 c^2 [(1/w6 - 1/2) + (1/w7 - 1/2)] d_x d_y phi / ((beta1 - beta2) phi)
    # to the extracted vorticity; with the literal sin sin scalar it dominates.
    pr, t, out, _, _ = tg_runs[(64, False)]
    _, _, wz, phi, dxy = tg_closed_form(64, 0.01, pr.nu, pr.diffusivity, t)
    raw = oracle.rel_l2(out["wz"], wz)
    w6, w7 = pr.omega_phi_hi[3], pr.omega_phi_hi[4]
    pred = -2.0 * pr.cs2phi * ((1.0 / w6 - 0.5) + (1.0 / w7 - 0.5)) * dxy / ((pr.beta1 - pr.beta2) * phi)
    corrected = oracle.rel_l2(out["wz"] - pred, wz)
    assert 5.0 < raw < 7.5
    assert corrected < 0.05


def test_fd_curl_agrees_on_smooth_field(tg_runs):
    e = []
    for n in (32, 64):
        _, _, out, _, _ = tg_runs[(n, True)]
        e.append(oracle.rel_l2(out["wz"], oracle.fd_curl(out["ux"], out["uy"])))
    assert e[1] < 1e-2
    assert e[0] / e[1] > 3.0


def test_mass_and_scalar_conservation(nthreads):
    vf = W.VortexField(L=64, n_blobs=16, sigma=4.0)
    pr = W.vortex_problem(64)
    o = oracle.Oracle(pr, nthreads=nthreads)
    f, g = o.init(*vf.fields())
    m0, s0 = f.sum(), g.sum()
    o.step(f, g, 200)
    assert abs(f.sum() - m0) / m0 < 1e-13
    assert abs(g.sum() - s0) / s0 < 1e-13


def test_mass_conserved_with_walls_and_lid(nthreads):
    pr = W.cavity_problem(24, 100.0, 0.1)
    o = oracle.Oracle(pr, nthreads=nthreads)
    f, g = o.init(*W.cavity_fields(24, 0.3))
    m0 = f.sum()
    o.step(f, g, 300)
    assert abs(f.sum() - m0) / m0 < 1e-13


def test_scalar_independent_of_beta(nthreads):
    # Sec. 3.1: the anisotropy sits in third-order equilibria and leaves the recovered
    # convection-diffusion equation unchanged.
    n = 32
    phis = []
    for b2 in (0.9, 1.0):
        o = oracle.Oracle(W.taylor_green_problem(n, beta2=b2), nthreads=nthreads)
        _, _, out = o.run(W.taylor_green_fields(n, 0.02), 300)
        phis.append(out["phi"] - 1.0)
    assert oracle.rel_l2(phis[0], phis[1]) < 2e-3


@pytest.mark.parametrize("umax,model", [(0.08, "mrt"), (0.01, "mrt"), (0.08, "srt"), (0.08, "central"), (0.08, "cascaded")])
def test_poiseuille_vorticity(umax, model, nthreads):
    # Sec. 5.1: 3 x 151, F = 3e-6, walls half-way (L = 75.5), phi 1 and 2 on the walls,
    # tau_phi = 0.57.  Started from the parabola; omega is linear in y.  The rows next to
    # the Dirichlet scalar walls are excluded: anti-bounce-back flips the even part of the
    # scalar's non-equilibrium there, which the extraction reads as an O(1) error.
    ny, F = 151, 3e-6
    L = ny / 2.0
    nu = F * L * L / (2.0 * umax)
    pr = W.channel_problem(3, ny, 0.5 + 3.0 * nu, 0.57, force=(F, 0.0), scalar_model=model)
    o = oracle.Oracle(pr, nthreads=nthreads)
    x, y = W.grid(3, ny)
    yc = y + 0.5 - L
    u = umax * (1.0 - yc * yc / (L * L))
    f, g = o.init(np.ones_like(u), u, 0.0 * u, 1.0 + (y + 0.5) / ny)
    # the parabola and the linear scalar are the steady state up to the wall slip; the
    # remaining transient decays on the viscous and diffusive time scales of the channel
    # (d_y phi is off by 1.4e-7 after 3000 steps, 1.3e-8 after 10k and 2e-9 after 30k)
    steps = 30000
    o.step(f, g, steps)
    out = o.extract(f, g, steps)
    wz = 2.0 * umax * yc / (L * L)
    # SRT over-relaxes the higher scalar moments (rate 1/tau_phi ~ 1.75), so the wall's
    # kinetic layer rings ~20 rows into the channel; MRT damps it within one row
    band = 25 if model == "srt" else 1
    inner = slice(band, ny - band)
    assert oracle.rel_l2(out["wz"][inner], wz[inner]) < 2e-3
    assert np.max(np.abs(out["dxuy"][inner])) < 2e-3 * np.max(np.abs(wz))
    # d_x u_x is zero in the closed form; what remains is the O(u d^2 u) term the
    # Chapman-Enskog relations of Sec. 2.1 drop
    assert np.max(np.abs(out["Sxx"][inner])) < 2e-3 * np.max(np.abs(wz))
    # scalar: linear profile between the half-way Dirichlet walls, exact gradient
    assert np.max(np.abs(out["phi"] - (1.0 + (y + 0.5) / ny))) < 1e-6
    assert np.max(np.abs(out["dyphi"] - 1.0 / ny)) < 1e-8


def test_couette_vorticity_and_moving_wall(nthreads):
    ny, U = 32, 0.02
    pr = W.channel_problem(3, ny, 0.9, 0.7, u_top=U, force_kind="none", phi_bottom=1.0, phi_top=2.0)
    o = oracle.Oracle(pr, nthreads=nthreads)
    x, y = W.grid(3, ny)
    f, g = o.init(np.ones_like(x), U * (y + 0.5) / ny, 0.0 * x, 1.0 + (y + 0.5) / ny)
    o.step(f, g, 20000)
    out = o.extract(f, g, 20000)
    assert np.max(np.abs(out["ux"] - U * (y + 0.5) / ny)) < 1e-7
    inner = slice(1, ny - 1)
    assert np.max(np.abs(out["wz"][inner] + U / ny)) < 1e-3 * U / ny
    assert np.max(np.abs(out["Sxy"] - 0.5 * U / ny)) < 1e-6 * U / ny


def test_fourroll_mill_re40(nthreads):
    # Sec. 5.2: 84^2, u0 = 0.035, Re = 2 pi u0 / nu = 40, phi = 2, tau_phi = 0.57.
    n, u0 = 84, 0.035
    nu_phys = u0 * 2.0 * math.pi / 40.0
    pr = W.fourroll_problem(n, nu_phys, u0)
    o = oracle.Oracle(pr, nthreads=nthreads)
    k = 2.0 * math.pi / n
    steps = int(3.0 / (pr.nu * k * k))
    f, g, out = o.run(W.fourroll_fields(n, u0), steps)
    x, y = W.grid(n, n)
    wz = -2.0 * u0 * k * np.sin(k * x) * np.cos(k * y)
    assert oracle.rel_l2(out["wz"], wz) < 2e-2


def test_fourroll_second_order_convergence(nthreads):
    # Sec. 5.2.1 reports slope -2.0 of E_g,omega.  Refinement at fixed tau and Reynolds
    # number (u0 ~ 1/N, diffusive scaling) gives it; with the paper's parameters read
    # literally (u0 fixed in lattice units, acoustic scaling) the error levels off near
    # 1 % from the O(u^2) terms the Chapman-Enskog relations drop.
    tau = 0.8
    nu = (tau - 0.5) / 3.0
    errs = []
    for n in (16, 32, 64):
        u0 = 0.04 * 16.0 / n
        k = 2.0 * math.pi / n
        pr = W.Problem(nx=n, ny=n, tau=tau, tau_phi=0.57, force_kind="fourroll",
                       force=(2.0 * nu * u0 * k * k, 0.0), force_k=k)
        o = oracle.Oracle(pr, nthreads=nthreads)
        steps = int(5.0 / (nu * k * k))
        _, _, out = o.run(W.fourroll_fields(n, u0), steps)
        x, y = W.grid(n, n)
        wz = -2.0 * u0 * k * np.sin(k * x) * np.cos(k * y)
        errs.append(oracle.rel_l2(out["wz"], wz))
    slopes = [math.log(errs[i + 1] / errs[i]) / math.log(2.0) for i in range(2)]
    assert all(-2.2 < s < -1.8 for s in slopes), slopes


def womersley(y, t, fm, omega, nu, L):
    """u and omega_z = -du/dy for F_x = F_m cos(Omega t) between walls at y = +-L,
    written with exp(-i Omega t) (the form that satisfies u_t = F + nu u_yy)."""
    gam = cmath.sqrt(1j * (L * L * omega / nu))
    A = 1j * fm / omega
    e = cmath.exp(-1j * omega * t)
    u = np.array([(A * (1.0 - cmath.cos(gam * yy / L) / cmath.cos(gam)) * e).real for yy in y])
    w = np.array([(-(A * (gam / L) * cmath.sin(gam * yy / L) / cmath.cos(gam)) * e).real for yy in y])
    return u, w


def test_womersley_pulsatile_flow(nthreads):
    # Sec. 5.3: 3 x 101, F_m = 1e-5, T = 10000, tau = 0.781 (Wo ~ 4).
    ny, fm, T, tau = 101, 1e-5, 10000, 0.781
    L = ny / 2.0
    om = 2.0 * math.pi / T
    pr = W.channel_problem(3, ny, tau, 0.57, force=(fm, 0.0), force_kind="pulsatile")
    pr = pr.with_(force_omega=om)
    o = oracle.Oracle(pr, nthreads=nthreads)
    x, y = W.grid(3, ny)
    yc = (y + 0.5 - L)[:, 0]
    u0, _ = womersley(yc, 0.0, fm, om, pr.nu, L)
    f, g = o.init(1.0, np.repeat(u0[:, None], 3, axis=1), 0.0, 1.0 + (y + 0.5) / ny)
    t = 0
    inner = slice(1, ny - 1)
    for target in (T + T // 4, T + T // 2, 2 * T):
        o.step(f, g, target - t, t)
        t = target
        out = o.extract(f, g, t)
        ua, wa = womersley(yc, t, fm, om, pr.nu, L)
        assert oracle.rel_l2(out["ux"][:, 1], ua) < 1e-2
        # omega = (2 N^phi - (b1 + b2) N) / (b1 - b2) multiplies the ~7e-4 relative lag of
        # N^phi in this unsteady flow by 2 / (b1 - b2) = 20
        assert oracle.rel_l2(out["wz"][inner, 1], wa[inner]) < 3e-2
        assert oracle.rel_l2(2.0 * out["Sxy"][inner, 1], -wa[inner]) < 2e-3


def test_unresolved_cavity_diverges_and_a_resolved_one_does_not():
    # tau -> 1/2 (Re 1e5 on 32^2 nodes, tau = 0.50029) is unstable: the state goes
    # non-finite within a few hundred steps; the same cavity at Re 100 stays bounded
    f0 = W.rest_fields(32, 32, 1.0, 0.5)
    bad = oracle.Oracle(W.cavity_problem(32, 1e5, 0.3, storage="f64"), nthreads=8).run(f0, 600)[2]
    good = oracle.Oracle(W.cavity_problem(32, 100.0, 0.3, storage="f64"), nthreads=8).run(f0, 600)[2]
    assert not np.isfinite(bad["ux"]).all()
    assert np.isfinite(good["ux"]).all() and np.abs(good["ux"]).max() < 0.5
