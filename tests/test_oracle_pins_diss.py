"""Pins of the oracle's control of the effective fluid-solid dissipation
(Sec. 2.2: the effective dissipative interaction between fluid and solid is
computed and controlled to impose no-slip or partial slip; the control's
form is the oracle's reading R6).

R6: for fluid i, E_i = sum over frozen j within r_c of w^D(r_ij), with
w^D = (1 - r/r_c)^2, is brought to T_i = eta rho_f W_D phi_i, where W_D is
the integral of w^D over the interaction sphere and phi_i the boundary
volume fraction; every fluid-solid pair of i uses gamma s_i and
sigma sqrt(s_i), s_i = T_i / E_i.

The cases below fix s_i and the forces by closed forms in which W_D comes
from numerical quadrature, not from the oracle's closed form, so a wrong
W_D, a missing phi, s applied to fluid-fluid pairs, or s instead of
sqrt(s) on the random force each fails a case.  CPU only.
"""
import numpy as np
import pytest
from scipy.integrate import quad

RC, RD, L = 1.0, 0.75, 10.0
ETA, RHO_F = 0.8, 6.0


def wc(r):
    return max(0.0, 1.0 - r / RC)


def w_d_integral():
    """Integral of w^D = w_c^2 over the sphere r < r_c, by quadrature."""
    v, err = quad(lambda r: 4.0 * np.pi * r * r * wc(r) ** 2, 0.0, RC, epsabs=1e-14, epsrel=1e-13)
    assert err < 1e-12
    return v


def params(orc, kT=1.0, gamma=4.5, A=-40.0, B=25.0, eta=ETA, search=0):
    return orc.make_params(box=L, A=A, B=B, gamma=gamma, rc=RC, rd=RD, kT=kT, wall_model=1,
                           diss_ctrl=eta, diss_rho=RHO_F, search=search)


def three():
    """Fluid i at the centre, frozen a at 0.3 along x, fluid b at 0.8 along y
    (|a - b| = sqrt(0.73) < r_c: b sees the frozen particle too)."""
    c = np.array([5.0, 5.0, 5.0])
    x = np.array([c, c + [0.3, 0.0, 0.0], c + [0.0, 0.8, 0.0]])
    return x, np.array([0, 1, 0], np.uint8)


def test_w_d_integral_is_two_pi_over_fifteen():
    assert w_d_integral() == pytest.approx(2.0 * np.pi / 15.0, rel=1e-13)


@pytest.mark.parametrize("search", [0, 1])
def test_scale_of_three_particles(orc, search):
    """s_i = eta rho_f W_D phi_i / E_i with phi_i = w1^2 / (w1^2 + w2^2) and
    E_i = w1^2, so s_i = eta rho_f W_D / (w1^2 + w2^2); the same for b with
    its own distances; frozen particles and a control that is off give 1."""
    x, fz = three()
    WD = w_d_integral()
    s = orc.diss_scale(params(orc, search=search), x, fz)
    rab = np.sqrt(0.3**2 + 0.8**2)
    exp_i = ETA * RHO_F * WD / (wc(0.3) ** 2 + wc(0.8) ** 2)
    exp_b = ETA * RHO_F * WD / (wc(rab) ** 2 + wc(0.8) ** 2)
    assert s[0] == pytest.approx(exp_i, rel=1e-13)
    assert s[2] == pytest.approx(exp_b, rel=1e-13)
    assert s[1] == 1.0
    # without phi the factor would be eta rho_f W_D / w1^2: far off
    assert abs(s[0] - ETA * RHO_F * WD / wc(0.3) ** 2) > 0.05 * s[0]
    assert np.all(orc.diss_scale(params(orc, eta=0.0), x, fz) == 1.0)


def test_fluid_without_frozen_neighbours_keeps_one(orc):
    """A fluid pair far from the solid: no fluid-solid pair, s = 1."""
    x = np.array([[2.0, 2.0, 2.0], [2.5, 2.0, 2.0], [8.0, 8.0, 8.0]])
    fz = np.array([0, 0, 1], np.uint8)
    assert np.all(orc.diss_scale(params(orc), x, fz) == 1.0)


def test_target_equals_eta_rho_wd_phi(orc):
    """The controlled fluid-solid weight s_i E_i equals eta rho_f W_D phi_i
    on a random cloud with a frozen slab (many neighbours of both kinds)."""
    rng = np.random.default_rng(3)
    x = rng.uniform(0.0, L, (900, 3))
    fz = (x[:, 1] < 2.5).astype(np.uint8)
    p = params(orc)
    s = orc.diss_scale(p, x, fz)
    phi = orc.phi(p, x, fz)
    WD = w_d_integral()
    d = x[:, None, :] - x[None, :, :]
    d -= L * np.round(d / L)
    r = np.sqrt((d**2).sum(-1))
    w2 = np.where((r < RC) & (r > 0.0), (1.0 - r / RC) ** 2, 0.0)
    E = (w2 * fz[None, :]).sum(1)
    fl = (fz == 0) & (E > 0)
    assert fl.sum() > 50
    np.testing.assert_allclose(s[fl] * E[fl], ETA * RHO_F * WD * phi[fl], rtol=1e-12)
    assert np.all(s[(fz == 0) & (E == 0)] == 1.0)


def test_dissipative_force_closed_form(orc):
    """kT = 0 (no noise), A = B = 0: only the dissipative force acts.
    F_i = -gamma s_i w1^2 (e_ia . v_i) e_ia - gamma w2^2 (e_ib . v_ib) e_ib:
    the fluid-solid pair carries s_i, the fluid-fluid pair does not."""
    x, fz = three()
    v = np.array([[0.7, -0.4, 0.3], [0.0, 0.0, 0.0], [-0.2, 0.5, 0.1]])
    g = 4.5
    p = params(orc, kT=0.0, A=0.0, B=0.0, gamma=g)
    rho = np.zeros(3)
    F, _, _ = orc.forces(p, x, v, np.zeros(3, np.int32), fz, rho, 0)
    WD = w_d_integral()
    s_i = ETA * RHO_F * WD / (wc(0.3) ** 2 + wc(0.8) ** 2)
    e_a = (x[0] - x[1]) / 0.3
    e_b = (x[0] - x[2]) / 0.8
    exp = -g * s_i * wc(0.3) ** 2 * np.dot(e_a, v[0]) * e_a - g * wc(0.8) ** 2 * np.dot(e_b, v[0] - v[2]) * e_b
    np.testing.assert_allclose(F[0], exp, rtol=1e-13, atol=1e-15)
    assert np.all(F[1] == 0.0)
    # the control off: the plain gamma on both pairs
    F0, _, _ = orc.forces(params(orc, kT=0.0, A=0.0, B=0.0, gamma=g, eta=0.0), x, v, np.zeros(3, np.int32), fz,
                          rho, 0)
    exp0 = -g * wc(0.3) ** 2 * np.dot(e_a, v[0]) * e_a - g * wc(0.8) ** 2 * np.dot(e_b, v[0] - v[2]) * e_b
    np.testing.assert_allclose(F0[0], exp0, rtol=1e-13, atol=1e-15)
    assert np.abs(F[0] - F0[0]).max() > 0.1


def test_random_force_takes_sqrt_of_scale(orc):
    """v = 0, A = B = 0: only the random force acts,
    F_i = sigma sqrt(s_i) w1 theta_ia / sqrt(dt) e_ia + sigma w2 theta_ib / sqrt(dt) e_ib,
    sigma = sqrt(2 gamma kT); theta from the pinned noise routine."""
    x, fz = three()
    g, kT, dt, step = 4.5, 1.0, 0.01, 7
    p = params(orc, kT=kT, A=0.0, B=0.0, gamma=g)
    F, _, _ = orc.forces(p, x, np.zeros((3, 3)), np.zeros(3, np.int32), fz, np.zeros(3), step)
    WD = w_d_integral()
    s_i = ETA * RHO_F * WD / (wc(0.3) ** 2 + wc(0.8) ** 2)
    sig = np.sqrt(2.0 * g * kT)
    e_a = (x[0] - x[1]) / 0.3
    e_b = (x[0] - x[2]) / 0.8
    th_a = orc.theta(p.seed, step, 0, 1)
    th_b = orc.theta(p.seed, step, 0, 2)
    exp = sig * np.sqrt(s_i) * wc(0.3) * th_a / np.sqrt(dt) * e_a + sig * wc(0.8) * th_b / np.sqrt(dt) * e_b
    np.testing.assert_allclose(F[0], exp, rtol=1e-13, atol=1e-14)
    # s instead of sqrt(s) would differ by (s_i - sqrt(s_i)) on the solid pair
    wrong = exp + sig * (s_i - np.sqrt(s_i)) * wc(0.3) * th_a / np.sqrt(dt) * e_a
    assert np.abs(wrong - F[0]).max() > 1e-3


def test_tangent_of_the_scale_by_finite_differences(orc):
    """The tangent of the force at creation (nsteps = 0, loss: virial
    pressure) of the three-particle system along a position direction equals
    central differences: the force on i moves with s_i, whose tangent the
    oracle takes through phi_i and E_i.  A state with A = B = 0 and kT = 0
    makes the dissipative force (and so s_i) the only pressure-free term, so
    the loss is the mean x-velocity after one step instead."""
    x, fz = three()
    v = np.array([[0.7, -0.4, 0.3], [0.0, 0.0, 0.0], [-0.2, 0.5, 0.1]])
    kw = dict(box=L, A=0.0, B=0.0, gamma=4.5, rc=RC, rd=RD, kT=0.0, wall_model=0, diss_ctrl=ETA,
              diss_rho=RHO_F)
    p = orc.make_params(**kw)
    t = np.zeros(3, np.int32)
    dx = np.array([[0.3, -0.2, 0.5], [0.1, 0.4, -0.3], [-0.6, 0.2, 0.1]])
    wts = (0.0, 0.0, 1.0)
    _, dL = orc.tangent(p, x, v, t, fz, 1, wts, False, dx0=dx)
    h = 1e-6
    fd = (orc.loss(p, x + h * dx, v, t, fz, 1, wts) - orc.loss(p, x - h * dx, v, t, fz, 1, wts)) / (2 * h)
    assert abs(dL - fd) <= 1e-6 * abs(fd) + 1e-10, (dL, fd)
    # the control's share: the same derivative without the control differs
    q = orc.make_params(**{**kw, "diss_ctrl": 0.0})
    _, d0 = orc.tangent(q, x, v, t, fz, 1, wts, False, dx0=dx)
    assert abs(dL - d0) > 1e-3 * abs(fd)
