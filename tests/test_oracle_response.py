"""Pins of the oracle's orbits, link responses, TDI and A, E, T (Eqs. 2.7-2.11)."""
import math

import numpy as np
import pytest

from oracle.orbits import Orbit, link_ends, LINK_LABELS
from oracle.phys import C_SI, YEAR_SI, ARM_SI, AU_SI
from oracle.response import Response, lagrange_weights, lagrange_offsets, k_u_v, cyclic, tdi_terms
from oracle.waveform import Template
from paper_2501_08261_amd import inputs


# ------------------------------------------------------------------ orbits
def test_static_orbit_exact():
    """P17: static arms: every light time is L/c and every side is L."""
    o = Orbit("static")
    for l in LINK_LABELS:
        assert np.all(o.light_time(l, np.array([0.0, 1e6])) == ARM_SI / C_SI)
        s, r = link_ends(l)
        d = np.linalg.norm(o.position(r, [0.0]) - o.position(s, [0.0]))
        assert d == pytest.approx(ARM_SI, rel=1e-14)
    c = sum(o.position(k, [0.0])[:, 0] for k in (1, 2, 3)) / 3
    assert np.allclose(c, [AU_SI, 0, 0], rtol=0, atol=1e-4)
    n = np.cross(o.position(2, [0.0])[:, 0] - o.position(1, [0.0])[:, 0],
                 o.position(3, [0.0])[:, 0] - o.position(1, [0.0])[:, 0])
    assert abs(n[2]) / np.linalg.norm(n) == pytest.approx(0.5, abs=1e-12)   # 60 deg inclination


def test_link_labels():
    assert [link_ends(l) for l in (1, 2, 3, -1, -2, -3)] == [(3, 2), (1, 3), (2, 1), (2, 3), (3, 1), (1, 2)]


def test_kepler_orbit_properties():
    """P17: period one year, arms near L and breathing, light-time equation solved."""
    o = Orbit("kepler")
    t = np.linspace(0, YEAR_SI, 97)
    for k in (1, 2, 3):
        assert np.allclose(o.position(k, t), o.position(k, t + YEAR_SI), rtol=0, atol=1e-3)
        r = np.linalg.norm(o.position(k, t), axis=0)
        assert np.all(np.abs(r / AU_SI - 1) < 1.01 * o.ecc)
    arms = []
    for l in LINK_LABELS:
        L = o.light_time(l, t)
        s, r = link_ends(l)
        res = L - np.linalg.norm(o.position(r, t) - o.position(s, t - L), axis=0) / C_SI
        assert np.max(np.abs(res)) < 1e-12
        assert np.all(np.abs(L * C_SI / ARM_SI - 1) < 0.02)
        arms.append(L)
    arms = np.array(arms)
    assert np.ptp(arms) > 1e-4                       # unequal and time-varying
    assert np.max(np.abs(arms[:, 0] - arms[:, -1])) < 1e-9   # periodic
    # Kepler with vanishing eccentricity: circular, rigid
    o0 = Orbit("kepler", arm=1.0)
    r = np.linalg.norm(o0.position(1, t), axis=0)
    assert np.allclose(r, AU_SI, rtol=1e-10)


# ----------------------------------------------------------- interpolation
@pytest.mark.parametrize("K", [2, 4, 6, 8, 16, 32])
def test_lagrange_exact_on_polynomials(K):
    """P23: K-tap Lagrange reproduces polynomials of degree < K; K = 2 is linear."""
    rng = np.random.default_rng(K)
    coef = rng.normal(size=K)
    frac = rng.uniform(0, 1, 50)
    o = lagrange_offsets(K)
    w = lagrange_weights(frac, K)
    vals = np.polyval(coef, o.astype(float))
    got = w @ vals
    want = np.polyval(coef, frac)
    scale = np.max(np.abs(w) @ np.abs(vals))   # condition of the weighted sum
    assert np.max(np.abs(got - want)) < 1e-13 * scale
    assert np.allclose(w.sum(-1), 1.0, atol=1e-12)
    if K == 2:
        assert np.allclose(w, np.stack([1 - frac, frac], -1), atol=1e-15)


# ------------------------------------------------------------- plane waves
def _plane_wave(f, amp=1e-20, psi_rot=0.0):
    w = 2 * math.pi * f

    def h(t):
        hp, hc = amp * np.cos(w * t), amp * 0.7 * np.sin(w * t + 0.3)
        c, s = math.cos(2 * psi_rot), math.sin(2 * psi_rot)
        return c * hp - s * hc, s * hp + c * hc
    return h


def _resp(hfun, orbit, gen=15, N=2048, dt=5.0, K=8, sky=(0.6, -0.4), t0=1e6):
    tpl = Template(np.r_[1e6, 7e5, np.zeros(6), 2e4, 0, 0, 0, sky[0], sky[1], 0, 0])
    return Response(tpl, t0, dt, N, orbit, taps=K, generation=gen, hfun=hfun, sky=sky)


def test_polarisation_rotation_invariance():
    """P14: rotating (u, v) by psi and (h+, hx) by 2 psi leaves y unchanged."""
    o = Orbit("kepler")
    t = np.linspace(1e6, 2e6, 7)
    r0 = _resp(_plane_wave(3e-3), o)
    y0 = [r0.y_exact(l, t) for l in LINK_LABELS]
    for psi in (0.3, 1.1, -2.0):
        r1 = _resp(_plane_wave(3e-3, psi_rot=psi), o)
        u, v = r0.u, r0.v
        # basis rotated by -psi while (h+, hx) rotate by +2 psi
        r1.u = math.cos(psi) * u - math.sin(psi) * v
        r1.v = math.sin(psi) * u + math.cos(psi) * v
        for l, y in zip(LINK_LABELS, y0):
            assert np.max(np.abs(r1.y_exact(l, t) - y)) < 1e-12 * np.max(np.abs(y))


def test_long_wavelength_limit():
    """P15: X_1.5 -> 2 (L/c)^2 [n12.h''.n12 - n13.h''.n13] as f L/c -> 0 (static arms),
    with a first-order relative error: err / (omega L) is the same constant at every f."""
    o = Orbit("static")
    L = ARM_SI / C_SI
    pos = {k: o.position(k, [0.0])[:, 0] for k in (1, 2, 3)}
    centre = sum(pos.values()) / 3
    n12 = (pos[2] - pos[1]) / ARM_SI
    n13 = (pos[3] - pos[1]) / ARM_SI
    ratios = []
    for f in (3e-6, 3e-5, 3e-4):
        hf = _plane_wave(f)
        r = _resp(hf, o, N=10 ** 7)
        idx = 1000 + np.linspace(0, 2 / (f * r.dt), 300).astype(np.int64)   # two full periods
        t = r.t0 + idx * r.dt
        X = r.xyz(idx, exact=True)[0]
        tc = t - 1.5 * L - r.k @ centre / C_SI
        w = 2 * math.pi * f
        e = 1e-3 / w
        hpp = [(a - 2 * b + c) / e ** 2 for a, b, c in zip(hf(tc + e), hf(tc), hf(tc - e))]

        def proj(n):
            un, vn = r.u @ n, r.v @ n
            return (un * un - vn * vn) * hpp[0] + 2 * un * vn * hpp[1]
        lw = 2 * L ** 2 * (proj(n12) - proj(n13))
        ratios.append(np.max(np.abs(X - lw)) / np.max(np.abs(lw)) / (w * L))
    assert max(ratios) < 1.0
    assert max(ratios) - min(ratios) < 0.01 * max(ratios)


class _Relabel:
    """Orbit seen with spacecraft renumbered: new k = old perm[k]."""

    def __init__(self, base, perm):
        self.base, self.perm = base, perm
        inv = {v: k for k, v in perm.items()}
        self.inv = inv

    def position(self, k, t):
        return self.base.position(self.perm[k], t)

    def light_time(self, l, t):
        s, r = link_ends(l)
        S, R = self.perm[s], self.perm[r]
        for ll in LINK_LABELS:
            if link_ends(ll) == (S, R):
                return self.base.light_time(ll, t)
        raise AssertionError


@pytest.mark.parametrize("gen", [15, 20])
def test_cyclic_relabelling(gen):
    """P19: Y(r1, r2, r3) = X(r2, r3, r1) and Z(r1, r2, r3) = X(r3, r1, r2), any orbit."""
    o = Orbit("kepler")
    idx = np.arange(800, 830)
    r = _resp(_plane_wave(7e-3), o, gen=gen)
    X, Y, Z = r.xyz(idx, exact=True)
    rY = _resp(_plane_wave(7e-3), _Relabel(o, {1: 2, 2: 3, 3: 1}), gen=gen)
    rZ = _resp(_plane_wave(7e-3), _Relabel(o, {1: 3, 2: 1, 3: 2}), gen=gen)
    s = np.max(np.abs(X))
    assert np.max(np.abs(rY.xyz(idx, exact=True)[0] - Y)) < 1e-12 * s
    assert np.max(np.abs(rZ.xyz(idx, exact=True)[0] - Z)) < 1e-12 * s


class _ConstDelays:
    """Static positions but arbitrary constant (unequal) light times."""

    def __init__(self, L):
        self.static, self.L = Orbit("static"), L

    def position(self, k, t):
        return self.static.position(k, t)

    def light_time(self, l, t):
        return np.full(np.atleast_1d(t).shape, self.L[l])


def test_tdi2_from_tdi15():
    """P18: with constant delays X_2(t) = X_1.5(t) - X_1.5(t - L2 - L-2 - L3 - L-3)."""
    rng = np.random.default_rng(3)
    L = {l: ARM_SI / C_SI * rng.uniform(0.9, 1.1) for l in LINK_LABELS}
    orb = _ConstDelays(L)
    idx = np.arange(900, 940)
    r2 = _resp(_plane_wave(4e-3), orb, gen=20)
    r15 = _resp(_plane_wave(4e-3), orb, gen=15)
    X2 = r2.xyz(idx, exact=True)[0]
    t = r15.t0 + idx * r15.dt
    D = L[2] + L[-2] + L[3] + L[-3]
    Xa = r15.xyz(idx, exact=True)[0]
    # X_1.5 at t - D: shift the grid origin so that output samples sit at t - D
    r15b = _resp(_plane_wave(4e-3), orb, gen=15, t0=r15.t0 - D)
    Xb = r15b.xyz(idx, exact=True)[0]
    assert np.max(np.abs(X2 - (Xa - Xb))) < 1e-10 * np.max(np.abs(X2))


def test_cyclic_label_map():
    assert [cyclic(l, 1) for l in (1, 2, 3, -1, -2, -3)] == [2, 3, 1, -2, -3, -1]
    assert len(tdi_terms(15, 0)) == 8 and len(tdi_terms(20, 2)) == 16


@pytest.mark.parametrize("orbit", ["static", "kepler"])
def test_interpolation_error_falls_with_taps(orbit):
    """P24: ORACLE-M converges to ORACLE-X (no interpolation) as K grows."""
    g = inputs.grid(4096, 5.0)
    p = inputs.tab1_injection(False, g, before_end=1000.0)
    tpl = Template(p)
    idx = np.arange(2500, 2560)
    errs = []
    for K in (2, 4, 8, 16):
        r = Response(tpl, g["t0"], g["dt"], g["n"], Orbit(orbit), taps=K, modes=((2, 2), (3, 3)),
                     generation=20)
        m = np.array(r.xyz(idx))
        x = np.array(r.xyz(idx, exact=True))
        errs.append(np.max(np.abs(m - x)) / np.max(np.abs(x)))
    # converges with K until the FP64 rounding floor of the phase (~1e-12 of h,
    # amplified by the TDI cancellation X/h ~ 1e-3) is reached
    assert errs[0] > 100 * errs[1] > 100 * errs[2]
    assert errs[2] < 1e-8 and errs[3] < 1e-8


def test_coarse_grid_closed_form():
    """N2: on the coarse grid an odd sample is the mean of its neighbours; for a sinusoid
    h = sin(w t) that is sin(w t) cos(w dt) exactly (and the even samples are untouched), which
    also gives the method's error (1 - cos(w dt)) ~ (w dt)^2 / 2."""
    w, dt, n = 0.07, 5.0, 101
    hfun = lambda t: (np.sin(w * t), np.cos(w * t))
    r = Response(None, 0.0, dt, n, Orbit("static"), hfun=hfun, sky=(0.3, 0.2), coarse=2)
    hp, hc = r.h_grid(np.arange(n))
    t = np.arange(n) * dt
    fac = np.where(np.arange(n) % 2 == 1, np.cos(w * dt), 1.0)
    assert np.max(np.abs(hp - np.sin(w * t) * fac)) < 1e-14
    assert np.max(np.abs(hc - np.cos(w * t) * fac)) < 1e-14
