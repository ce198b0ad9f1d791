"""Pins of the oracle's quaternion / Wigner-D twist-up (Eqs. 2.1-2.6)."""
import math

import numpy as np
import pytest

from oracle import twist as tw
from oracle.waveform import Template, MODES_ALL

RNG = np.random.default_rng(20250108)


def _Y_closed(l, m, th, ph):
    """Textbook closed forms of -2Y_lm (LAL convention)."""
    c, s = math.cos(th / 2), math.sin(th / 2)
    e = np.exp(1j * m * ph)
    pi = math.pi
    table = {
        (2, 2): math.sqrt(5 / (64 * pi)) * (1 + math.cos(th)) ** 2,
        (2, 1): math.sqrt(5 / (16 * pi)) * math.sin(th) * (1 + math.cos(th)),
        (2, 0): math.sqrt(15 / (32 * pi)) * math.sin(th) ** 2,
        (2, -1): math.sqrt(5 / (16 * pi)) * math.sin(th) * (1 - math.cos(th)),
        (2, -2): math.sqrt(5 / (64 * pi)) * (1 - math.cos(th)) ** 2,
        (3, 3): -math.sqrt(21 / (2 * pi)) * c ** 5 * s,
        (3, 2): math.sqrt(7 / (4 * pi)) * c ** 4 * (3 * math.cos(th) - 2),
        (3, -2): math.sqrt(7 / (4 * pi)) * s ** 4 * (3 * math.cos(th) + 2),
        (3, -3): math.sqrt(21 / (2 * pi)) * c * s ** 5,
        (4, 4): 3 * math.sqrt(7 / pi) * c ** 6 * s ** 2,
        (4, -4): 3 * math.sqrt(7 / pi) * c ** 2 * s ** 6,
    }
    return table[(l, m)] * e


@pytest.mark.parametrize("lm", [(2, 2), (2, 1), (2, 0), (2, -1), (2, -2), (3, 3), (3, 2), (3, -2),
                                (3, -3), (4, 4), (4, -4)])
def test_W_matches_textbook_harmonics(lm):
    """P7: sqrt((2l+1)/4pi) W^l_m(q(phi, iota, 0)) = -2Y_lm(iota, phi)."""
    l, m = lm
    for _ in range(20):
        th, ph = RNG.uniform(0, math.pi), RNG.uniform(0, 2 * math.pi)
        Qa, Qb = tw.Q_ab(tw.quat_from_euler(ph, th, 0.0))
        got = math.sqrt((2 * l + 1) / (4 * math.pi)) * tw.W_lm(l, m, Qa, Qb)
        assert abs(got - _Y_closed(l, m, th, ph)) < 2e-15


def test_quaternion_special_cases():
    """P8: |q| = 1; beta = 0 gives Q_a = exp(i(a+g)/2), Q_b = 0 and W^l_m = delta_m2 exp(2i(a+g))."""
    for _ in range(20):
        a, b, g = RNG.uniform(-7, 7, 3)
        assert np.linalg.norm(tw.quat_from_euler(a, b, g)) == pytest.approx(1.0, abs=1e-15)
        Qa, Qb = tw.Q_ab(tw.quat_from_euler(a, 0.0, g))
        assert abs(Qa - np.exp(0.5j * (a + g))) < 1e-15 and abs(Qb) < 1e-15
        for l in (2, 3, 4):
            for m in range(-l, l + 1):
                want = np.exp(2j * (a + g)) if m == 2 else 0.0
                assert abs(tw.W_lm(l, m, Qa, Qb) - want) < 1e-14


def test_W_unitarity():
    """P9: sum_m |D^l_{m,2}|^2 = 1 for any unit quaternion."""
    for _ in range(20):
        q = RNG.normal(size=4)
        q /= np.linalg.norm(q)
        Qa, Qb = tw.Q_ab(q)
        for l in (2, 3, 4, 5):
            tot = sum(abs(tw.W_lm(l, m, Qa, Qb)) ** 2 for m in range(-l, l + 1))
            assert tot == pytest.approx(1.0, abs=1e-14)


def test_quaternion_matrix_homomorphism():
    """P12: R(q1 q2) = R(q1) R(q2) and q(a, b, g) maps to R_z(a) R_y(b) R_z(g)."""
    for _ in range(20):
        a1, b1, g1, a2, b2, g2 = RNG.uniform(-4, 4, 6)
        q1, q2 = tw.quat_from_euler(a1, b1, g1), tw.quat_from_euler(a2, b2, g2)
        R1 = tw.rot_z(a1) @ tw.rot_y(b1) @ tw.rot_z(g1)
        R2 = tw.rot_z(a2) @ tw.rot_y(b2) @ tw.rot_z(g2)
        assert np.allclose(tw.quat_to_matrix(q1), R1, atol=1e-14)
        assert np.allclose(tw.quat_to_matrix(tw.quat_mul(q1, q2)), R1 @ R2, atol=1e-14)
        assert np.allclose(tw.quat_to_matrix(tw.quat_conj(q1)), R1.T, atol=1e-14)


def _p(chi1, chi2, m1=1e6, m2=7e5):
    p = np.zeros(16)
    p[0], p[1] = m1, m2
    p[2:5], p[5:8] = chi1, chi2
    p[8], p[9], p[10], p[14] = 2e4, 2.6, 4.0, 0.4
    return p


def test_zero_inplane_spin_reduces_to_aligned():
    """P10: precessing path with zero in-plane spins equals the aligned path."""
    tpl = Template(_p((0, 0, 0.6), (0, 0, -0.3)))
    t = np.linspace(tpl.t_start * 0.99, 200 * tpl.Ms, 3000)
    a = tw.polarizations(tpl, t, MODES_ALL, precessing=False)
    b = tw.polarizations(tpl, t, MODES_ALL, precessing=True)
    s = np.max(np.abs(a[0]))
    assert np.max(np.abs(a[0] - b[0])) < 1e-14 * s and np.max(np.abs(a[1] - b[1])) < 1e-14 * s


def test_composite_rotation_identity_at_reference():
    """P11: at f_ref the CP -> L0 rotation is a pure z-rotation (here the identity)."""
    tpl = Template(_p((0.3, 0.4, 0.5), (-0.2, 0.1, 0.3)))
    pr = tw.Precession(tpl)
    t_ref = -5.0 * tpl.Ms / (tpl.eta * tpl.theta_ref ** 8)
    al, be, ga, _ = pr.angles(np.array([t_ref]))
    q = tw.quat_mul(pr.q_J_L0(), tw.quat_from_euler(al, be, ga))[0]
    assert abs(q[1]) < 1e-12 and abs(q[2]) < 1e-12
    assert abs(abs(q[0]) - 1.0) < 1e-12
    # beta at f_ref is the angle between L and J
    assert be[0] == pytest.approx(pr.beta_ref, abs=1e-12)


@pytest.mark.parametrize("seed", range(4))
def test_explicit_equals_single_sum(seed):
    """P13: explicit Eqs. (2.1)-(2.3) equal the single-sum Eq. (2.4) (precessing)."""
    rng = np.random.default_rng(seed)
    c1 = rng.normal(size=3)
    c1 *= rng.uniform(0.1, 0.95) / np.linalg.norm(c1)
    c2 = rng.normal(size=3)
    c2 *= rng.uniform(0.1, 0.95) / np.linalg.norm(c2)
    p = _p(c1, c2, m1=rng.uniform(3e5, 3e6), m2=rng.uniform(1e5, 3e5))
    p[9], p[10], p[14] = rng.uniform(0, math.pi), rng.uniform(0, 2 * math.pi), rng.uniform(0, math.pi)
    tpl = Template(p)
    t = np.linspace(tpl.t_start * 0.9, 100 * tpl.Ms, 400)
    a = tw.polarizations(tpl, t, MODES_ALL, precessing=True)
    b = tw.polarizations_explicit(tpl, t, MODES_ALL, precessing=True)
    s = np.max(np.abs(b[0]))
    assert np.max(np.abs(a[0] - b[0])) < 1e-13 * s and np.max(np.abs(a[1] - b[1])) < 1e-13 * s


def test_precession_modulates():
    """Sanity: in-plane spin makes the precessing and aligned waveforms differ."""
    tpl = Template(_p((0.5, 0.3, 0.2), (0.0, 0.0, 0.0)))
    t = np.linspace(tpl.t_start * 0.5, -10 * tpl.Ms, 2000)
    a = tw.polarizations(tpl, t, MODES_ALL, precessing=False)
    b = tw.polarizations(tpl, t, MODES_ALL, precessing=True)
    assert np.max(np.abs(a[0] - b[0])) > 1e-2 * np.max(np.abs(a[0]))
