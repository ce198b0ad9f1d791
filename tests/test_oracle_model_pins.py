"""Pins of the oracle's builder-defined model pieces against published closed forms.

The paper names the IMRPhenomT family and NNLO precession angles but prints
none of their formulas (Sec. II.A), so the oracle defines a PhenomT-form
model from public post-Newtonian physics.  These tests fix each of its parts
against results that do not come from the oracle itself:

* P31  mode amplitude ratios: the mode sum equals the textbook 0.5PN and 1PN
       polarisations of a quasi-circular binary;
* P32  2PN TaylorT3 phase: its frequency evolution agrees with the
       energy-balance equation built from the published 2PN energy and flux
       (with the 1.5PN spin-orbit terms) through O(x^2);
* P33  remnant and (2,2,0) ringdown fits: test-particle and equal-mass limits,
       and the Kerr quasi-normal frequencies of Leaver's continued fraction;
* P34  precession angles: gamma obeys the minimal-rotation condition
       d gamma/dt = -cos(beta) d alpha/dt to the order the model keeps;
* P16  link response and TDI 1.5 for a monochromatic plane wave on static
       equal arms: the one-way Doppler from the photon line integral, and
       Michelson X as (1 - D^2) times the difference of the two round trips.

Each test also plants a plausible mistake in the oracle (on the CPU) and
checks that the pin catches it.
"""
import math

import numpy as np
import pytest

from oracle import response as oresp
from oracle import twist
from oracle import waveform as owf
from oracle.orbits import Orbit, link_ends, LINK_LABELS
from oracle.phys import ARM_SI, C_SI, MPC_SI
from oracle.response import Response, k_u_v
from oracle.waveform import Template, MODES_ALL


def _params(m1, m2, c1=(0.0, 0.0, 0.0), c2=(0.0, 0.0, 0.0), iota=1.0, phi=0.0, D=2e4):
    p = np.zeros(16)
    p[0], p[1] = m1, m2
    p[2:5], p[5:8] = c1, c2
    p[8], p[9], p[10] = D, iota, phi
    return p


# ------------------------------------------------------------- P31 mode ratios
def _pn_polarisation_error(tpl, iota):
    """Largest |h - h_PN| / (2 M eta x / D) over inspiral samples, at Phi = pi/2.

    h: the oracle's aligned-spin polarisations (modes 22, 21, 33, 32, 44) plus the
    three leading modes the model leaves out, taken from the same published
    multipole expansion: the 1PN correction of h22, and h31, h42.  h_PN: the
    textbook quasi-circular polarisations through 1PN (oscillating terms; the
    non-oscillating memory term of the m = 0 modes is in neither side), with
    psi the orbital phase, c = cos iota, s = sin iota, Delta = (m1 - m2)/M:
      H+ = -(1+c^2) cos 2psi
           - x^1/2 s Delta [(5/8 + c^2/8) cos psi - 9/8 (1+c^2) cos 3psi]
           + x [((19 + 9c^2 - 2c^4) - eta (19 - 11c^2 - 6c^4))/6 cos 2psi
                - 4/3 s^2 (1+c^2)(1-3eta) cos 4psi]
      Hx = -2c sin 2psi - 3/4 x^1/2 s c Delta [sin psi - 3 sin 3psi]
           + x [c/3 ((17 - 4c^2) - eta (13 - 12c^2)) sin 2psi - 8/3 (1-3eta) c s^2 sin 4psi]
    """
    eta, dl = tpl.eta, tpl.delta
    c, s = math.cos(iota), math.sin(iota)
    t = -np.geomspace(min(3e6, -0.9 * tpl.t_start), 2.0 * tpl.T, 9)    # after the f_low start
    x = tpl.x_of_t(t)
    ps = 0.5 * tpl.phi22(t)
    hp, hc = twist.polarizations(tpl, t + tpl.tc, MODES_ALL)
    pref = 2.0 * tpl.Ms * C_SI * eta * x / (tpl.DL * MPC_SI)

    def pair(l, m, H):
        h = pref * math.sqrt(16.0 * math.pi / 5.0) * H * np.exp(-1j * m * ps)
        return h * twist.sYlm_m2(l, m, iota, tpl.phi_ref) + \
            (-1) ** l * np.conj(h) * twist.sYlm_m2(l, -m, iota, tpl.phi_ref)
    extra = pair(2, 2, x * (-107.0 / 42.0 + 55.0 * eta / 42.0)) \
        + pair(3, 1, 1j * dl / (12.0 * math.sqrt(14.0)) * np.sqrt(x)) \
        + pair(4, 2, math.sqrt(5.0) / 63.0 * (1.0 - 3.0 * eta) * x)
    hp, hc = hp + extra.real, hc - extra.imag
    Hp = (-(1 + c * c) * np.cos(2 * ps)
          - np.sqrt(x) * s * dl * ((5 / 8 + c * c / 8) * np.cos(ps) - 9 / 8 * (1 + c * c) * np.cos(3 * ps))
          + x * (((19 + 9 * c * c - 2 * c ** 4) - eta * (19 - 11 * c * c - 6 * c ** 4)) / 6 * np.cos(2 * ps)
                 - 4 / 3 * s * s * (1 + c * c) * (1 - 3 * eta) * np.cos(4 * ps)))
    Hc = (-2 * c * np.sin(2 * ps)
          - 0.75 * s * c * dl * np.sqrt(x) * (np.sin(ps) - 3 * np.sin(3 * ps))
          + x * (c / 3 * ((17 - 4 * c * c) - eta * (13 - 12 * c * c)) * np.sin(2 * ps)
                 - 8 / 3 * (1 - 3 * eta) * c * s * s * np.sin(4 * ps)))
    return max(np.max(np.abs(hp - pref * Hp) / pref), np.max(np.abs(hc - pref * Hc) / pref))


IOTAS = (0.3, 1.1, 2.0, 2.9)


def test_mode_ratios_match_pn_polarisations():
    """P31: at the line-of-sight azimuth Phi = pi/2 of the textbook expansion the mode
    sum reproduces the 0.5PN and 1PN polarisations to rounding (x up to 0.1)."""
    for m1, m2 in ((8e5, 3e5), (5e5, 5e5), (9e6, 1e6)):
        for iota in IOTAS:
            tpl = Template(_params(m1, m2, iota=iota, phi=0.5 * math.pi))
            assert _pn_polarisation_error(tpl, iota) < 1e-13


@pytest.mark.parametrize("plant", ["h21 sign", "h33 sign", "h32 sqrt(7/5)", "h44 eta", "h33 real"])
def test_mode_ratio_pin_catches_mistakes(plant, monkeypatch):
    real = owf.Template.mode_ratio

    def wrong(self, l, m, x):
        v = real(self, l, m, x)
        if plant == "h21 sign" and (l, m) == (2, 1):
            return -v
        if plant == "h33 sign" and (l, m) == (3, 3):
            return -v
        if plant == "h32 sqrt(7/5)" and (l, m) == (3, 2):
            return v * 7.0 / 5.0
        if plant == "h44 eta" and (l, m) == (4, 4):
            return v * (1.0 - 2.0 * self.eta) / (1.0 - 3.0 * self.eta)
        if plant == "h33 real" and (l, m) == (3, 3):
            return 1j * v
        return v
    monkeypatch.setattr(owf.Template, "mode_ratio", wrong)
    errs = [_pn_polarisation_error(Template(_params(8e5, 3e5, iota=i, phi=0.5 * math.pi)), i) for i in IOTAS]
    assert max(errs) > 1e-4


# ------------------------------------------------------ P32 energy balance
def _balance_dxdt(tpl, x):
    """dx/dt = -F / (dE/dx) from the published 2PN energy and flux of a
    quasi-circular binary with aligned spins (spin-orbit terms at 1.5PN), x = (M omega)^(2/3):
      E = -(M eta x / 2) [1 - (3/4 + eta/12) x + (14/3 S_l + 2 Delta Sigma_l) x^3/2
                          + (-27/8 + 19 eta/8 - eta^2/24) x^2]
      F = 32/5 eta^2 x^5 [1 - (1247/336 + 35 eta/12) x + (4 pi - 4 S_l - 5/4 Delta Sigma_l) x^3/2
                          + (-44711/9072 + 9271 eta/504 + 65 eta^2/18) x^2]
    with S_l = (m1/M)^2 chi1 + (m2/M)^2 chi2 and Sigma_l = (m2/M) chi2 - (m1/M) chi1."""
    eta, dl = tpl.eta, tpl.delta
    Sl = tpl.m1f ** 2 * tpl.chi1l + tpl.m2f ** 2 * tpl.chi2l
    Sg = tpl.m2f * tpl.chi2l - tpl.m1f * tpl.chi1l
    e2, e3, e4 = -0.75 - eta / 12.0, 14.0 / 3.0 * Sl + 2.0 * dl * Sg, -27.0 / 8.0 + 19.0 * eta / 8.0 - eta ** 2 / 24.0
    f2 = -1247.0 / 336.0 - 35.0 * eta / 12.0
    f3 = 4.0 * math.pi - 4.0 * Sl - 1.25 * dl * Sg
    f4 = -44711.0 / 9072.0 + 9271.0 * eta / 504.0 + 65.0 * eta ** 2 / 18.0
    dEdx = -0.5 * eta * tpl.Ms * (1 + 2 * e2 * x + 2.5 * e3 * x ** 1.5 + 3 * e4 * x ** 2)
    F = 32.0 / 5.0 * eta ** 2 * x ** 5 * (1 + f2 * x + f3 * x ** 1.5 + f4 * x ** 2)
    return -F / dEdx


def _model_dxdt(tpl, x):
    out = []
    for xv in x:
        th = tpl.solve_theta(xv ** 1.5 / tpl.Ms)
        w = tpl.omega_orb_theta(th)
        dw = tpl.domega_orb_dtheta(th) * tpl.dtheta_dt(th)
        out.append(2.0 / 3.0 * (tpl.Ms * w) ** (2.0 / 3.0) / w * dw)
    return np.array(out)


def _x2_coefficient(tpl):
    """Fit r(x) = model/balance - 1 as x^2 (c4 + c5 x^1/2 + c6 x) on x in [1e-5, 1e-3];
    a model consistent through 2PN has c4 = 0 (its first disagreement is at 2.5PN)."""
    xs = np.geomspace(1e-5, 1e-3, 13)
    r = _model_dxdt(tpl, xs) / _balance_dxdt(tpl, xs) - 1.0
    A = np.stack([np.ones_like(xs), np.sqrt(xs), xs], 1)
    return np.linalg.lstsq(A, r / xs ** 2, rcond=None)[0], r


PN_CASES = [(6e5, 4e5, 0.0, 0.0), (9e5, 1e5, 0.9, -0.5), (5e5, 5e5, -0.8, 0.7), (9.1e6, 9.1e5, 0.99, 0.99)]


@pytest.mark.parametrize("case", PN_CASES)
def test_taylort3_matches_energy_balance(case):
    """P32: the model's frequency evolution equals the energy balance through 2PN;
    the residual is O(x^5/2) (log-slope 2.5 between x = 1e-4 and 1e-3)."""
    m1, m2, c1, c2 = case
    tpl = Template(_params(m1, m2, (0, 0, c1), (0, 0, c2)))
    c, r = _x2_coefficient(tpl)
    assert abs(c[0]) < 5e-3
    slope = math.log10(abs(_model_dxdt(tpl, [1e-3])[0] / _balance_dxdt(tpl, np.array([1e-3]))[0] - 1)
                       / abs(_model_dxdt(tpl, [1e-4])[0] / _balance_dxdt(tpl, np.array([1e-4]))[0] - 1))
    assert 2.35 < slope < 2.65
    assert np.max(np.abs(r)) < 5e-6


@pytest.mark.parametrize("plant", ["a2 eta", "a3 pi", "spin-orbit sign", "a4 constant", "a4 eta^2"])
def test_energy_balance_pin_catches_mistakes(plant):
    worst = 0.0
    for m1, m2, c1, c2 in PN_CASES[1:]:
        tpl = Template(_params(m1, m2, (0, 0, c1), (0, 0, c2)))
        beta = sum((113.0 / 12.0 * mf ** 2 + 25.0 / 4.0 * tpl.eta) * ch
                   for mf, ch in ((tpl.m1f, tpl.chi1l), (tpl.m2f, tpl.chi2l)))
        if plant == "a2 eta":
            tpl.a2 += 0.01 * 55.0 / 96.0 * tpl.eta
        elif plant == "a3 pi":
            tpl.a3 -= 1e-3 * 0.75 * math.pi
        elif plant == "spin-orbit sign":
            tpl.a3 -= 2.0 * 3.0 / 16.0 * beta
        elif plant == "a4 constant":
            tpl.a4 *= 1.01
        else:
            tpl.a4 -= 1855.0 / 2048.0 * tpl.eta ** 2
        worst = max(worst, abs(_x2_coefficient(tpl)[0][0]))
    assert worst > 2e-2


# ------------------------------------------------ P33 remnant and ringdown
# Kerr (2,2,0) frequencies M omega = omega_R - i omega_I from Leaver's continued fraction
# (published tables), at dimensionless spins a = 0, 0.5, 0.9
LEAVER_220 = ((0.0, 0.37367, 0.08896), (0.5, 0.46412, 0.08564), (0.9, 0.67161, 0.06486))


def test_qnm_fit_against_leaver():
    """P33: the ringdown frequency and quality factor Q = omega_R / (2 omega_I) of the
    model's fit lie within the fit's few-per-cent accuracy of the published values."""
    for a, wr, wi in LEAVER_220:
        w, q = owf._qnm22(a)
        assert w == pytest.approx(wr, rel=0.02)
        assert q == pytest.approx(wr / (2.0 * wi), rel=0.03)


def test_remnant_fit_limits():
    """P33: remnant spin -> 2 sqrt(3) eta + chi1 as eta -> 0 (a test particle plunging from
    the Schwarzschild ISCO carries L = 2 sqrt(3) mu M); equal-mass non-spinning remnant of
    numerical relativity: a_f = 0.6865, M_f / M = 0.9516."""
    for eta in (1e-6, 1e-5):
        m1f = 0.5 * (1 + math.sqrt(1 - 4 * eta))
        af, _ = owf._remnant(eta, m1f, 1 - m1f, 0.0, 0.0)
        assert af / eta == pytest.approx(2.0 * math.sqrt(3.0), rel=1e-4)
        af, _ = owf._remnant(eta, m1f, 1 - m1f, 0.6, 0.0)
        assert af == pytest.approx(0.6, abs=1e-4)
    af, mf = owf._remnant(0.25, 0.5, 0.5, 0.0, 0.0)
    assert af == pytest.approx(0.6865, abs=2e-3)
    assert mf == pytest.approx(0.9516, abs=1e-3)


def test_ringdown_pin_catches_mistakes(monkeypatch):
    real = owf._qnm22
    monkeypatch.setattr(owf, "_qnm22", lambda a: (1.5251 - 1.1568 * (1.0 - a) ** 0.2, real(a)[1]))
    with pytest.raises(AssertionError):
        test_qnm_fit_against_leaver()
    monkeypatch.setattr(owf, "_qnm22", lambda a: (real(a)[0], 0.7 + 1.4187 * (1.0 - a) ** -0.4))
    with pytest.raises(AssertionError):
        test_qnm_fit_against_leaver()
    monkeypatch.setattr(owf, "_qnm22", real)
    r = owf._remnant
    monkeypatch.setattr(owf, "_remnant", lambda eta, a, b, c, d: (r(eta, a, b, c, d)[0] - 0.1 * eta, r(eta, a, b, c, d)[1]))
    with pytest.raises(AssertionError):
        test_remnant_fit_limits()


# ------------------------------------------------- P34 minimal rotation
SPINS = (((0.5, 0.2, 0.6), (0.1, -0.3, 0.2)), ((0.9, 0.0, 0.1), (0.0, 0.0, 0.0)),
         ((-0.3, 0.6, -0.5), (0.4, 0.4, 0.4)))


def _minimal_rotation_excess(pr):
    """max over u of |gamma' + cos(beta) alpha'| / |alpha'| divided by the order the model
    drops, |sigma| vsigma^2 u^3 + vsigma^4 u^4 (derivatives in u by central differences)."""
    u = np.array([0.01, 0.02, 0.05, 0.1, 0.2])
    h = 1e-6 * u
    da = (pr.a_of_u(u + h) - pr.a_of_u(u - h)) / (2 * h)
    dg = (pr.g_of_u(u + h) - pr.g_of_u(u - h)) / (2 * h)
    res = np.abs(dg + da * pr.cos_beta(u)) / np.abs(da)
    return float(np.max(res / (abs(pr.sig) * pr.vsig ** 2 * u ** 3 + pr.vsig ** 4 * u ** 4)))


def test_minimal_rotation_gamma():
    """P34: with u = (M omega22/2)^(1/3) the precession angles satisfy the minimal-rotation
    condition gamma' = -cos(beta) alpha' up to terms of relative order sigma vsigma^2 u^3
    and vsigma^4 u^4 (the model keeps the leading vsigma^2 u^2 correction of gamma)."""
    for c1, c2 in SPINS:
        pr = twist.Precession(Template(_params(1e6, 3e5, c1, c2)))
        assert _minimal_rotation_excess(pr) < 1.0


@pytest.mark.parametrize("plant", ["vsigma term dropped", "vsigma sign", "u^-3 coefficient"])
def test_minimal_rotation_pin_catches_mistakes(plant, monkeypatch):
    def wrong(self, u):
        if plant == "vsigma term dropped":
            return 2.0 * self.C * (u ** -3 / 3.0 + 0.5 * self.sig * u ** -2)
        if plant == "vsigma sign":
            return 2.0 * self.C * (u ** -3 / 3.0 + 0.5 * self.sig * u ** -2 + 0.5 * self.vsig ** 2 / u)
        return 2.0 * self.C * (u ** -3 / 2.0 + 0.5 * self.sig * u ** -2 - 0.5 * self.vsig ** 2 / u)
    monkeypatch.setattr(twist.Precession, "g_of_u", wrong)
    pr = twist.Precession(Template(_params(1e6, 3e5, *SPINS[0])))
    assert _minimal_rotation_excess(pr) > 3.0


# --------------------------------------- P16 plane wave, static equal arms
F_PW, A_PW, B_PW, PH_PW = 0.02, 1e-20, 0.7e-20, 0.3
SKY = (0.6, -0.4)


def _pw(t):
    w = 2 * math.pi * F_PW
    return A_PW * np.cos(w * t), B_PW * np.sin(w * t + PH_PW)


def _pw_dot(t):
    w = 2 * math.pi * F_PW
    return -A_PW * w * np.sin(w * t), B_PW * w * np.cos(w * t + PH_PW)


def _y_photon(orbit, l, t):
    """One-way Doppler of link l at reception times t: -1/2 the integral of
    n.(d h/dt).n along the unperturbed photon path x(t') = r_s + c n (t' - t + L),
    h_ij = h+ (uu - vv)_ij + hx (uv + vu)_ij evaluated at the retarded argument
    t' - k.x(t')/c; 48-point Gauss-Legendre quadrature over the flight time."""
    k, u, v = k_u_v(*SKY)
    s, r = link_ends(l)
    rs, rr = orbit.position(s, [0.0])[:, 0], orbit.position(r, [0.0])[:, 0]
    L = np.linalg.norm(rr - rs) / C_SI
    n = (rr - rs) / np.linalg.norm(rr - rs)
    xg, wg = np.polynomial.legendre.leggauss(48)
    te = np.asarray(t, dtype=np.float64) - L
    tp = te[:, None] + 0.5 * L * (xg[None, :] + 1.0)
    hp_d, hc_d = _pw_dot(tp - (k @ rs) / C_SI - (k @ n) * (tp - te[:, None]))
    un, vn = u @ n, v @ n
    return -0.25 * L * (((un * un - vn * vn) * hp_d + 2.0 * un * vn * hc_d) @ wg)


def _x_closed(orbit, t):
    """Michelson X for equal arms: (1 - D^2) [(y_-2 + D y_2) - (y_3 + D y_-3)], D the
    delay by L = arm/c; link 2 runs 1 -> 3 and -2 back, link -3 runs 1 -> 2 and 3 back."""
    L = ARM_SI / C_SI

    def rt(tt):
        return (_y_photon(orbit, -2, tt) + _y_photon(orbit, 2, tt - L)) - \
            (_y_photon(orbit, 3, tt) + _y_photon(orbit, -3, tt - L))
    return rt(t) - rt(t - 2 * L)


def _resp(K):
    tpl = Template(np.r_[1e6, 7e5, np.zeros(6), 2e4, 0, 0, 0, SKY[0], SKY[1], 0, 0])
    return Response(tpl, 0.0, 5.0, 4096, Orbit("static"), taps=K, generation=15, hfun=_pw, sky=SKY)


IDX = np.arange(200, 4000, 37)


def _p16_errors(K=32):
    o = Orbit("static")
    r = _resp(K)
    t = r.t0 + IDX * r.dt
    ey = max(np.max(np.abs(_y_photon(o, l, t) - r.y_exact(l, t))) / np.max(np.abs(r.y_exact(l, t)))
             for l in LINK_LABELS)
    Xc = _x_closed(o, t)
    ex = np.max(np.abs(r.xyz(IDX, exact=True)[0] - Xc)) / np.max(np.abs(Xc))
    return ey, ex, Xc


def test_plane_wave_closed_form():
    """P16: at f L/c = 0.17 (far from the long-wavelength limit) the oracle's link responses
    (Eq. 2.8) equal the photon line integral and its TDI 1.5 X (Eq. 2.9) the factorised
    Michelson form, to the FP64 rounding of the absolute times (1e-12); the K-tap
    method converges to it as K grows."""
    ey, ex, Xc = _p16_errors()
    assert ey < 1e-11 and ex < 1e-11
    prev = 1.0
    for K in (2, 4, 8, 16, 32):
        r = _resp(K)
        e = np.max(np.abs(r.xyz(IDX)[0] - Xc)) / np.max(np.abs(Xc))
        assert e < 0.1 * prev or e < 1e-11
        prev = e
    assert prev < 1e-11


@pytest.mark.parametrize("plant", ["x+ half dropped", "sender/receiver swapped", "delay dropped", "term sign"])
def test_plane_wave_pin_catches_mistakes(plant, monkeypatch):
    if plant == "x+ half dropped" or plant == "sender/receiver swapped":
        real = oresp.Response.link_geometry

        def wrong(self, l, tau):
            pp, pc, t_s, t_r = real(self, l, tau)
            if plant == "x+ half dropped":
                return 2.0 * pp, pc, t_s, t_r
            return pp, pc, t_r, t_s
        monkeypatch.setattr(oresp.Response, "link_geometry", wrong)
    else:
        x15 = list(oresp.X15)
        sg, l, dl = x15[1]
        x15[1] = (sg, l, ()) if plant == "delay dropped" else (-sg, l, dl)
        monkeypatch.setattr(oresp, "X15", tuple(x15))
    ey, ex, _ = _p16_errors()
    assert max(ey, ex) > 1e-3
