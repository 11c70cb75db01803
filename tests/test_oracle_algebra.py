"""Pins of the oracle's moment algebra, equilibria, collision and extraction.

Each test checks the oracle against something other than itself: matrices
printed in the paper, textbook D2Q9 values, closed-form product equilibria,
exact conservation laws, or the forward Chapman-Enskog relations of Sec. 2.1
and Sec. 3.1 (which the extraction of Sec. 4 must invert).
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from conftest import golden

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=float)
CS2 = 1.0 / 3.0


def d1q3(u):
    """1D three-velocity equilibrium weights for velocities (0, +1, -1) with c_s^2 = 1/3."""
    return {0: 2.0 / 3.0 - u * u, 1: (CS2 + u * u + u) / 2.0, -1: (CS2 + u * u - u) / 2.0}


def product_equilibrium(rho, ux, uy):
    """Textbook D2Q9 equilibrium as the tensor product of two D1Q3 equilibria."""
    wx, wy = d1q3(ux), d1q3(uy)
    return np.array([rho * wx[int(EX[a])] * wy[int(EY[a])] for a in range(9)])


def test_bare_inverse_matches_app_b():
    T, Tinv, P, Pinv = oracle.matrices()
    printed = golden("app_b_bare_inverse.txt") / 4.0
    assert np.allclose(Pinv, printed, atol=1e-15, rtol=0)


def test_natural_inverse_matches_app_b_via_moment_relation():
    # natural moments m = M q with m3 = q_xx + q_yy, m4 = q_xx - q_yy (Sec. 2 vs App. B)
    T, Tinv, P, Pinv = oracle.matrices()
    M = np.eye(9)
    M[3, 3], M[3, 4], M[4, 3], M[4, 4] = 1.0, 1.0, 1.0, -1.0
    printed = golden("app_b_bare_inverse.txt") / 4.0
    assert np.allclose(Tinv, printed @ np.linalg.inv(M), atol=1e-15, rtol=0)
    assert np.allclose(T @ Tinv, np.eye(9), atol=1e-15)


def test_rest_equilibrium_is_d2q9_weights():
    o = oracle.Oracle(W.taylor_green_problem(4))
    f, g = o.init(1.0, 0.0, 0.0, 1.0)
    w = golden("d2q9_weights.txt") / 36.0
    assert np.allclose(f[:, 0, 0], w, atol=1e-16, rtol=0)
    assert np.allclose(g[:, 0, 0], w, atol=1e-16, rtol=0)


@pytest.mark.parametrize("seed", range(5))
def test_fluid_equilibrium_is_product_form(seed):
    r = np.random.default_rng(seed)
    rho, ux, uy = 1.0 + 0.2 * r.standard_normal(), 0.1 * r.standard_normal(), 0.1 * r.standard_normal()
    o = oracle.Oracle(W.taylor_green_problem(4))
    f, g = o.init(rho, ux, uy, rho)
    assert np.allclose(f[:, 0, 0], product_equilibrium(rho, ux, uy), atol=1e-15, rtol=0)


@pytest.mark.parametrize("seed", range(5))
def test_scalar_equilibrium_anisotropy(seed):
    # beta1 = beta2 = 1: same product form with rho -> phi.  beta != 1 adds only the
    # third-order columns of the printed App. B inverse, times (beta - 1) c^2 phi u.
    r = np.random.default_rng(100 + seed)
    phi, ux, uy = 1.0 + r.random(), 0.1 * r.standard_normal(), 0.1 * r.standard_normal()
    b1, b2 = 1.0 + 0.3 * r.random(), 1.0 - 0.3 * r.random()
    iso = oracle.Oracle(W.taylor_green_problem(4, beta1=1.0, beta2=1.0))
    ani = oracle.Oracle(W.taylor_green_problem(4, beta1=b1, beta2=b2))
    _, g_iso = iso.init(1.0, ux, uy, phi)
    _, g_ani = ani.init(1.0, ux, uy, phi)
    assert np.allclose(g_iso[:, 0, 0], product_equilibrium(phi, ux, uy), atol=1e-15, rtol=0)
    Pinv = golden("app_b_bare_inverse.txt") / 4.0
    expect = (b1 - 1.0) * CS2 * phi * uy * Pinv[:, 6] + (b2 - 1.0) * CS2 * phi * ux * Pinv[:, 7]
    assert np.allclose(g_ani[:, 0, 0] - g_iso[:, 0, 0], expect, atol=1e-15, rtol=0)


def _random_state(seed, amp=0.02):
    r = np.random.default_rng(seed)
    o = oracle.Oracle(W.taylor_green_problem(4))
    f, g = o.init(1.0 + 0.1 * r.random(), 0.05 * r.standard_normal(), 0.05 * r.standard_normal(), 1.0 + r.random())
    return f[:, 0, 0] + amp * r.standard_normal(9), g[:, 0, 0] + amp * r.standard_normal(9)


@pytest.mark.parametrize("model", ["mrt", "srt", "cascaded", "central"])
def test_collision_invariants(model):
    # mass and scalar are collision invariants; momentum is conserved without force
    # and gains exactly F per step with the trapezoidal source (Sec. 2).
    pr = W.taylor_green_problem(4, tau=0.63, tau_phi=0.77, omega3=1.3, scalar_model=model,
                                omega_hi=(1.1, 1.2, 0.9), omega_phi_hi=(1.05, 0.95, 1.15, 1.25, 1.35, 1.45))
    o = oracle.Oracle(pr)
    for seed in range(4):
        f, g = _random_state(seed)
        for F in ((0.0, 0.0), (1e-3, -2e-3)):
            fs, gs = o.collide_node(f, g, F)
            assert abs(fs.sum() - f.sum()) < 1e-15
            assert abs(gs.sum() - g.sum()) < 1e-15
            assert abs((fs * EX).sum() - (f * EX).sum() - F[0]) < 1e-15
            assert abs((fs * EY).sum() - (f * EY).sum() - F[1]) < 1e-15


@pytest.mark.parametrize("seed", range(8))
def test_source_moments_have_central_moments_of_a_pure_force(seed):
    # Sec. 2, the sigma' list: the raw source moments are those of a source whose central
    # moments about u are (0, F_x, F_y, 0, ..., 0), i.e. it adds momentum F and nothing
    # else in the frame moving with the fluid.  Mapped to populations with the inverse
    # pinned by App. B, the central moments are taken here by their definition, so a
    # wrong, dropped or swapped term in any of the nine entries shows up.
    r = np.random.default_rng(200 + seed)
    Fx, Fy = r.standard_normal(2)
    ux, uy = 0.2 * r.standard_normal(2)
    _, Tinv, _, _ = oracle.matrices()
    s = Tinv @ oracle.source_moments(Fx, Fy, ux, uy)
    cx, cy = EX - ux, EY - uy
    orders = [(0, 0), (1, 0), (0, 1), (2, 0), (0, 2), (1, 1), (2, 1), (1, 2), (2, 2)]
    got = np.array([np.sum(s * cx ** p * cy ** q) for p, q in orders])
    expect = np.array([0.0, Fx, Fy, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0])
    assert np.max(np.abs(got - expect)) < 1e-15 * max(1.0, abs(Fx), abs(Fy))
    # and a force-free source is zero
    assert np.array_equal(oracle.source_moments(0.0, 0.0, ux, uy), np.zeros(9))


def test_equilibrium_is_fixed_point():
    o = oracle.Oracle(W.taylor_green_problem(4, omega3=1.4))
    f, g = o.init(1.1, 0.04, -0.03, 1.7)
    fs, gs = o.collide_node(f[:, 0, 0], g[:, 0, 0])
    assert np.allclose(fs, f[:, 0, 0], atol=1e-15, rtol=0)
    assert np.allclose(gs, g[:, 0, 0], atol=1e-15, rtol=0)


def test_srt_equals_mrt_with_uniform_scalar_rates():
    # App. B: the SRT scheme relaxes every population at 1/tau_phi, which is MRT with
    # Lambda^phi = I / tau_phi on the same equilibria.
    tp = 0.73
    srt = oracle.Oracle(W.taylor_green_problem(4, tau_phi=tp, scalar_model="srt"))
    mrt = oracle.Oracle(W.taylor_green_problem(4, tau_phi=tp, scalar_model="mrt", omega_phi_hi=(1.0 / tp,) * 6))
    for seed in range(4):
        f, g = _random_state(seed)
        assert np.allclose(srt.collide_node(f, g)[1], mrt.collide_node(f, g)[1], atol=1e-15, rtol=0)


def test_cascaded_basis_reading_matches_printed_updates():
    K = np.empty((9, 9))
    oracle.lib().orc_cascaded_basis(K.ctypes.data_as(oracle.C.POINTER(oracle.C.c_double)))
    assert np.array_equal(K, golden("app_c_population_updates.txt"))


def test_cascaded_equals_noncascaded_central_moments():
    # App. C and App. D relax the same central moments at the same rates, so the two
    # printed algorithms must give one post-collision state.
    hi = (0.9, 0.95, 1.1, 1.2, 1.3, 1.4)
    c = oracle.Oracle(W.taylor_green_problem(4, scalar_model="cascaded", omega_phi_hi=hi))
    d = oracle.Oracle(W.taylor_green_problem(4, scalar_model="central", omega_phi_hi=hi))
    for seed in range(6):
        f, g = _random_state(seed, amp=0.05)
        assert np.allclose(c.collide_node(f, g)[1], d.collide_node(f, g)[1], atol=2e-15, rtol=0)


def _manufactured(pr, rho, ux, uy, phi, A, grad_phi, F):
    """Populations whose non-equilibrium moments are the Chapman-Enskog ones
    (Sec. 2.1, eqs. strainratexxpyy/xxmyy/xy; Sec. 3.1, eqs. 1stnoneqmmomentx/y_CDE and
    offdiagonal2ndnoneqmmoment_CDE) for a chosen velocity gradient A[i][j] = d_j u_i."""
    o = oracle.Oracle(pr)
    T, Tinv, _, _ = oracle.matrices()
    lf, lg = o.lam_f, o.lam_g
    c2, cp2, b1, b2 = pr.cs2, pr.cs2phi, pr.beta1, pr.beta2
    dxux, dyux, dxuy, dyuy = A[0][0], A[0][1], A[1][0], A[1][1]
    px, py = grad_phi
    m1 = np.zeros(9)
    m1[3] = -2.0 * c2 * rho / lf[3] * (dxux + dyuy)
    m1[4] = -2.0 * c2 * rho / lf[4] * (dxux - dyuy)
    m1[5] = -c2 * rho / lf[5] * (dxuy + dyux)
    n1 = np.zeros(9)
    n1[1] = -cp2 * px / lg[1]
    n1[2] = -cp2 * py / lg[2]
    n1[5] = -cp2 / lg[5] * (phi * (b1 * dxuy + b2 * dyux) + (b1 * uy * px + b2 * ux * py))
    S = oracle.source_moments(F[0], F[1], ux, uy)
    mbar = oracle.meq_fluid(rho, ux, uy, c2) + m1 - 0.5 * S
    n = oracle.neq_scalar(phi, ux, uy, cp2, b1, b2) + n1
    return o, Tinv @ mbar, Tinv @ n


@pytest.mark.parametrize("seed", range(6))
def test_extraction_inverts_chapman_enskog_relations(seed):
    r = np.random.default_rng(seed)
    pr = W.taylor_green_problem(4, tau=0.55 + 0.5 * r.random(), tau_phi=0.55 + 0.5 * r.random(),
                                omega3=0.8 + 0.6 * r.random(), beta1=1.0 + 0.2 * r.random(),
                                beta2=0.8 + 0.1 * r.random(), omega_phi_hi=(1.0, 1.0, 0.7 + 0.6 * r.random(), 1.0, 1.0, 1.0))
    rho, ux, uy, phi = 1.0 + 0.05 * r.standard_normal(), 0.05 * r.standard_normal(), 0.05 * r.standard_normal(), 0.5 + r.random()
    A = 1e-3 * r.standard_normal((2, 2))
    gp = 1e-3 * r.standard_normal(2)
    F = 1e-5 * r.standard_normal(2)
    o, f, g = _manufactured(pr, rho, ux, uy, phi, A, gp, F)
    out = o.extract_node(f, g, F)
    tol = 1e-15
    assert abs(out["rho"] - rho) < tol and abs(out["phi"] - phi) < tol
    assert abs(out["ux"] - ux) < tol and abs(out["uy"] - uy) < tol
    assert abs(out["Sxx"] - A[0][0]) < 1e-13
    assert abs(out["Syy"] - A[1][1]) < 1e-13
    assert abs(out["Sxy"] - 0.5 * (A[0][1] + A[1][0])) < 1e-13
    assert abs(out["dxuy"] - A[1][0]) < 1e-12
    assert abs(out["dyux"] - A[0][1]) < 1e-12
    assert abs(out["wz"] - (A[1][0] - A[0][1])) < 1e-12
    assert abs(out["dxphi"] - gp[0]) < 1e-13 and abs(out["dyphi"] - gp[1]) < 1e-13
    # Q = -S_ij S_ij / 2 + w^2 / 4 and the Lamb vector w x u (Sec. 1)
    Sm = 0.5 * (A + A.T)
    w = A[1][0] - A[0][1]
    assert abs(out["Q"] - (-0.5 * np.sum(Sm * Sm) + 0.25 * w * w)) < 1e-15
    assert abs(out["R"] - np.trace(Sm @ Sm @ Sm) / 3.0) < 1e-15
    assert abs(out["Lx"] - (-w * uy)) < 1e-15 and abs(out["Ly"] - w * ux) < 1e-15


@pytest.mark.parametrize("seed", [3, 4, 5])
def test_invariants_and_lamb_vector_by_matrix_identities(seed):
    # Sec. 1 defines Q, R and L for the 3D velocity gradient A_ij = d_j u_i.  Checked here
    # through identities other than the formulas the extraction evaluates: R through the
    # eigenvalues of S (the omega term vanishes in the plane), Q through -tr(A A) / 2 of the
    # 3x3 gradient of a divergence-free state, L through a 3D cross product.
    r = np.random.default_rng(seed)
    pr = W.taylor_green_problem(4, tau=0.6 + 0.3 * r.random(), tau_phi=0.6 + 0.3 * r.random())
    rho, ux, uy, phi = 1.0 + 0.05 * r.standard_normal(), 0.05 * r.standard_normal(), 0.05 * r.standard_normal(), 1.0
    for traceless in (True, False):
        A = 1e-3 * r.standard_normal((2, 2))
        if traceless:
            A[1][1] = -A[0][0]
        o, f, g = _manufactured(pr, rho, ux, uy, phi, A, np.zeros(2), np.zeros(2))
        out = o.extract_node(f, g, np.zeros(2))
        lam = np.linalg.eigvalsh(0.5 * (A + A.T))
        assert abs(out["R"] - np.sum(lam ** 3) / 3.0) < 1e-15
        G = np.zeros((3, 3))
        G[:2, :2] = A
        Om = 0.5 * (G - G.T)
        if traceless:
            assert abs(out["Q"] - (-0.5 * np.trace(G @ G))) < 1e-15
            assert abs(out["R"]) < 1e-15                        # = -det(G) of a plane flow
        assert abs(out["Q"] - (-0.5 * np.sum(lam ** 2) + 0.5 * np.sum(Om * Om))) < 1e-15
        wvec = np.array([G[2][1] - G[1][2], G[0][2] - G[2][0], G[1][0] - G[0][1]])   # curl u
        L = np.cross(wvec, np.array([ux, uy, 0.0]))
        assert abs(out["Lx"] - L[0]) < 1e-15 and abs(out["Ly"] - L[1]) < 1e-15 and L[2] == 0.0


def test_uniform_flow_has_no_gradient():
    o = oracle.Oracle(W.taylor_green_problem(8))
    f, g = o.init(1.0, 0.03, -0.02, 1.5)
    o.step(f, g, 20)
    out = o.extract(f, g, 20)
    for k in ("Sxx", "Syy", "Sxy", "wz", "dxuy", "dyux", "dxphi", "dyphi"):
        assert np.max(np.abs(out[k])) < 1e-15, k


def test_phi_mask():
    o = oracle.Oracle(W.taylor_green_problem(4, phi_min=1e-3))
    f, g = o.init(1.0, 0.01, 0.0, 1e-4)
    out = o.extract(f, g)
    assert np.all(np.isnan(out["wz"])) and np.all(np.isnan(out["dxuy"]))
    assert np.all(np.isfinite(out["Sxy"]))
