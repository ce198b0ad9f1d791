"""Pins of the oracle's PhenomT-form waveform against closed forms and invariants."""
import math

import numpy as np
import pytest

from oracle.waveform import Template, cp_modes, MODES_ALL
from oracle import twist
from paper_2501_08261_amd import inputs


def _params(m1=1e6, m2=7e5, c1=(0, 0, 0.7), c2=(0, 0, 0.4), D=2e4, iota=2.6, phi=4.0, psi=0.0):
    p = np.zeros(16)
    p[0], p[1] = m1, m2
    p[2:5], p[5:8] = c1, c2
    p[8], p[9], p[10], p[14] = D, iota, phi, psi
    return p


CASES = [(6.6667e5, 3.3333e5, 0.5, 0.3), (1e6, 7e5, 0.7, 0.4), (9.09e6, 9.09e5, -0.99, -0.99),
         (5e4, 5e4, 0.99, 0.99), (9.09e4, 9.09e3, 0.99, -0.99), (3e5, 2e5, -0.5, 0.9)]


def test_leading_order_closed_form():
    """P1: with PN terms off, phi_orb = -theta^-5/eta + const, omega = theta^3/(8M),
    which in terms of t is phi_orb(t) = -(1/eta) [eta (-t)/(5M)]^(5/8) + const."""
    tpl = Template(_params(), pn=False)
    t = -np.geomspace(1e7, 1.2 * tpl.T, 200)
    M, eta = tpl.Ms, tpl.eta
    closed = -(1.0 / eta) * (eta * (-t) / (5.0 * M)) ** 0.625
    phi = 0.5 * tpl.phi22(t)
    dphi = phi - closed
    assert np.max(np.abs(dphi - dphi[0])) < 1e-9 * np.max(np.abs(closed))
    th = (eta * (-t) / (5.0 * M)) ** -0.125
    assert np.allclose(0.5 * tpl.omega22(t), th ** 3 / (8.0 * M), rtol=1e-14, atol=0)


@pytest.mark.parametrize("pn", [False, True])
def test_phase_derivative_is_frequency(pn):
    """P1: d phi22 / dt = omega22 (inspiral and merger), by central differences."""
    tpl = Template(_params(), pn=pn)
    for t in np.concatenate([-np.geomspace(5e6, 1.05 * tpl.T, 40), np.linspace(0.95 * tpl.t_m, 20 * tpl.Ms, 40)]):
        h = 1e-3 * tpl.Ms
        d = (tpl.phi22(np.array([t + h])) - tpl.phi22(np.array([t - h])))[0] / (2 * h)
        w = tpl.omega22(np.array([t]))[0]
        assert abs(d - w) < 1e-6 * w


@pytest.mark.parametrize("case", CASES)
def test_frequency_monotone_and_peak_at_zero(case):
    """P2, P3: omega22 strictly increasing on the whole signal; |h22| maximal at t = 0."""
    m1, m2, c1, c2 = case
    tpl = Template(_params(m1, m2, (0, 0, c1), (0, 0, c2)))
    assert tpl.valid
    t = np.concatenate([np.linspace(tpl.t_start, 2 * tpl.t_m, 20000, endpoint=False),
                        np.linspace(2 * tpl.t_m, 0.0, 20000, endpoint=False),
                        np.linspace(0.0, 300 * tpl.Ms, 20001)])
    assert np.all(np.diff(tpl.omega22(t)) > 0)
    A = tpl.amp22(t)
    assert t[np.argmax(A)] == 0.0
    h = 1e-4 * tpl.Ms
    A0 = tpl.amp22(np.array([-h, 0.0, h]))
    assert A0[1] > A0[0] and A0[1] > A0[2]


@pytest.mark.parametrize("case", CASES)
def test_c1_continuity_at_matching(case):
    """P5: omega, phase and amplitude are C^1 across t_m (and A across t = 0)."""
    m1, m2, c1, c2 = case
    tpl = Template(_params(m1, m2, (0, 0, c1), (0, 0, c2)))
    for f in (tpl.omega22, tpl.phi22, tpl.amp22):
        for tj in (tpl.t_m, 0.0):
            e = 1e-7 * tpl.Ms
            v = f(np.array([tj - e, tj + e]))
            scale = abs(f(np.array([tj]))[0]) + 1e-300
            assert abs(v[1] - v[0]) < 1e-8 * scale
            e2 = 1e-5 * tpl.Ms
            left = (f(np.array([tj - e2]))[0] - f(np.array([tj - 3 * e2]))[0]) / (2 * e2)
            right = (f(np.array([tj + 3 * e2]))[0] - f(np.array([tj + e2]))[0]) / (2 * e2)
            slope = (f(np.array([tj + e2]))[0] - f(np.array([tj - e2]))[0]) / (2 * e2)
            assert abs(left - right) < 1e-3 * (abs(slope) + abs(left)) + 1e-6 * scale / tpl.Ms


def test_equal_chirp_mass_equal_phase():
    """P6: at leading order (PN terms off) the phase depends only on the chirp mass."""
    Mc = 5e5
    out = []
    for eta in (0.25, 0.2, 0.12):
        M = Mc / eta ** 0.6
        d = math.sqrt(1 - 4 * eta)
        tpl = Template(_params(M * (1 + d) / 2, M * (1 - d) / 2), pn=False)
        out.append(tpl)
    t = -np.geomspace(5e6, 5e4, 100)
    ref = out[0].phi22(t)
    for tpl in out[1:]:
        assert np.max(np.abs(tpl.phi22(t) - ref)) < 1e-9 * np.max(np.abs(ref))


def test_mode_symmetry_reflection():
    """P4: h_{l,-m} = (-1)^l conj(h_lm) makes iota -> pi - iota conjugate h (aligned spins)."""
    g = inputs.grid(4096, 5.0)
    p = _params(iota=0.7, phi=1.3)
    p[11] = inputs.peak_time(g, 1000.0)
    t = g["t0"] + np.arange(g["n"]) * g["dt"]
    a = twist.polarizations(Template(p), t, MODES_ALL)
    p2 = p.copy()
    p2[9] = math.pi - p[9]
    b = twist.polarizations(Template(p2), t, MODES_ALL)
    s = np.max(np.abs(a[0]))
    assert np.max(np.abs(a[0] - b[0])) < 1e-13 * s
    assert np.max(np.abs(a[1] + b[1])) < 1e-13 * s


def test_hard_start_and_reference():
    """Modes vanish before the f_low start and the orbital phase is zero at f_ref."""
    tpl = Template(_params(m1=6e6, m2=2e6))
    t = tpl.tc + np.linspace(tpl.t_start - 5e4, tpl.t_start + 5e4, 1001)
    h = cp_modes(tpl, t)
    before = t - tpl.tc < tpl.t_start
    assert np.all(h[:, before] == 0) and np.all(np.abs(h[0, ~before]) > 0)
    f22 = tpl.omega22(np.array([tpl.t_start]))[0] / (2 * math.pi)
    assert f22 == pytest.approx(1e-4, rel=1e-12)
    assert 0.5 * tpl.phi22(np.array([tpl.t_start]))[0] == pytest.approx(0.0, abs=1e-9)


def test_leading_amplitude():
    """|h22| = 8 sqrt(pi/5) eta (M/D) x in the inspiral (x = (M omega22/2)^(2/3))."""
    tpl = Template(_params())
    t = np.array([-4e6, -1e6, -2e5])
    x = (tpl.Ms * tpl.omega22(t) / 2) ** (2 / 3)
    Mm = tpl.Ms * 299792458.0
    D = 2e4 * 3.085677581491367e22
    want = 8 * math.sqrt(math.pi / 5) * tpl.eta * Mm / D * x
    h = cp_modes(tpl, t + tpl.tc, ((2, 2),))
    assert np.allclose(np.abs(h[0]), want, rtol=1e-13)


def test_unphysical_flagged():
    assert not Template(_params(c1=(0, 0, 1.2))).valid
    assert not Template(_params(D=-1)).valid
    assert not Template(_params(m1=1e9, m2=1e9)).valid
