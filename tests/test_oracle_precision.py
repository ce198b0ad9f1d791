"""P35: the FP64 rounding floor of the method, measured on the oracle alone.

The oracle evaluates the same model (same FP64 coefficients and inputs) in x87
extended precision (np.longdouble, 64-bit significand) when its Template and
Response are built with real=np.longdouble: every per-template constant, the
phase, the sample and delayed times, the Euler angles and the interpolation
weights then carry 11 more bits.  The difference FP64 - extended is the FP64
oracle's own rounding error, which any FP64 implementation of the method
shares in size (not in sign): the phase is the difference of two ~1e4 rad
values (the orbital phase at t and at f_ref) and the sample times reach
n dt, so one FP64 rounding of either moves h by ~1e-12 of itself.

These measurements are what the parity tolerances of the GPU tests rest on:
* logL (one-day (2,2) case): the FP64 oracle misses the extended reference by
  up to ~5e-5 = 5e-12 (d|d), above the 1e-6 absolute target, so the GPU is
  compared with the extended reference at 1e-6 + 1e-11 (d|d);
* TDI 2.0 at 2^20 samples: a 1e7 Msun template's channels sit (2 pi f L)^2
  below h, and the FP64 oracle's own error reaches ~2e-8 of the channel
  (~1.5e-11 of max|h|), above the 1e-9 relative target; the GPU is compared
  with the extended reference at 1e-9 of the channel plus the time-rounding
  floor 32 u n min(2 omega dt, pi) max|h| (u = 2^-53).
"""
import math

import numpy as np
import pytest

from oracle import likelihood as olk
from oracle.orbits import Orbit
from oracle.response import Response
from oracle.waveform import Template, MODES_ALL
from paper_2501_08261_amd import inputs

U64 = 2.0 ** -53


def _aet(p, g, real, taps, orbit="static", modes=((2, 2),), precessing=False, gen=15, idx=None):
    r = Response(Template(p, real=real), g["t0"], g["dt"], g["n"], Orbit(orbit), taps=taps, modes=modes,
                 precessing=precessing, generation=gen, real=real)
    if idx is None:
        r.cache_full_grid()
        idx = np.arange(g["n"])
    return np.array([np.asarray(a, dtype=np.float64) for a in r.aet(idx)]), r


def test_extended_reference_phase_accuracy():
    """The extended evaluation is accurate well below the FP64 floor: the (2,2) inspiral phase
    of the one-day case, 2 (Phi(theta(t)) - Phi(theta_ref)), recomputed at 40 digits (mpmath,
    with the model's FP64 coefficients as exact binary numbers and theta_ref solved to full
    precision), agrees with the extended oracle to ~1e-15 rad, while the FP64 oracle is off
    by ~1e-12 rad.  This checks the arithmetic of the reference, not the model."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 40
    g, inj, _ = inputs.single_template_case()
    t = g["t0"] + np.arange(0, g["n"] - 400, 997) * g["dt"]     # inspiral samples (t < t_m)
    tpl = Template(inj)
    m1, m2 = mp.mpf(inj[0]), mp.mpf(inj[1])
    M = m1 + m2
    Ms = M * mp.mpf(4.925490947641267e-06)
    eta = m1 * m2 / M ** 2
    a2 = mp.mpf(3715.0 / 8064.0) + mp.mpf(55.0 / 96.0) * eta
    m1f, m2f = m1 / M, m2 / M
    beta = sum((mp.mpf(113.0 / 12.0) * mf ** 2 + mp.mpf(25.0 / 4.0) * eta) * mp.mpf(c)
               for mf, c in ((m1f, inj[4]), (m2f, inj[7])))
    a3 = mp.mpf(-0.75 * math.pi) + mp.mpf(3.0 / 16.0) * beta
    a4 = mp.mpf(9275495.0 / 14450688.0) + mp.mpf(284875.0 / 258048.0) * eta + mp.mpf(1855.0 / 2048.0) * eta ** 2

    def Phi(th):
        return -(th ** -5) / eta * (1 + a2 * th ** 2 + a3 * th ** 3 + a4 * th ** 4)

    def w_orb(th):
        return th ** 3 / (8 * Ms) * (1 + mp.mpf(0.6) * a2 * th ** 2 + mp.mpf(0.4) * a3 * th ** 3
                                     + mp.mpf(0.2) * a4 * th ** 4)
    th_ref = mp.findroot(lambda th: w_orb(th) - mp.mpf(math.pi * 1e-4), mp.mpf(tpl.theta_ref))
    want = [2 * (Phi((eta * (mp.mpf(inj[11]) - mp.mpf(ti)) / (5 * Ms)) ** mp.mpf(-0.125)) - Phi(th_ref))
            for ti in t]
    got = {}
    for real in (np.float64, np.longdouble):
        tp = Template(inj, real=real)
        tt = real(g["t0"]) + np.arange(0, g["n"] - 400, 997).astype(real) * real(g["dt"])
        ph = tp.phi22(tt - tp.tc)
        got[real] = max(abs(float(mp.mpf(str(ph[i])) - want[i])) for i in range(len(want)))
    assert got[np.longdouble] < 1e-14
    assert got[np.float64] > 1e-13


def test_loglike_fp64_floor_one_day():
    """The logL tolerance on the oracle alone: at the one-day (2,2) case (K = 2 and 8) the FP64 oracle's logL
    differs from the extended reference by more than the 1e-6 absolute target for the
    mismatched template, and by less than 1e-11 (d|d), the bound the GPU tests apply."""
    g, inj, tmpl = inputs.single_template_case()
    S = olk.channel_psds(g["n"], g["dt"], 15)
    for taps in (2, 8):
        d64, _ = _aet(inj, g, np.float64, taps)
        h64, _ = _aet(tmpl, g, np.float64, taps)
        dld, _ = _aet(inj, g, np.longdouble, taps)
        hld, _ = _aet(tmpl, g, np.longdouble, taps)
        dd = olk.noise_inner(dld, S, g["dt"])
        gaps = [abs(a - b) for a, b in zip(olk.loglike(d64, h64, S, g["dt"]), olk.loglike(dld, hld, S, g["dt"]))]
        gap_inj = abs(olk.loglike(d64, d64, S, g["dt"])[0] - olk.loglike(dld, dld, S, g["dt"])[0])
        assert max(gaps) > 1e-6                       # FP64 itself cannot meet 1e-6 absolute here
        assert max(gaps + [gap_inj]) < 1e-11 * dd     # the 1e-6 + 1e-11 (d|d) tolerance covers it
        assert max(gaps) > 1e-12 * dd                 # and is not loose by orders of magnitude


def test_tdi2_fp64_floor_heavy_template():
    """The long-grid TDI tolerance on the oracle alone: the bench batch's heaviest template (1e7 Msun, precessing,
    Kepler arms, TDI 2.0, K = 8, 2^20 samples): the FP64 oracle's own error on the last
    samples exceeds 1e-9 of the channel, and stays below the time-rounding floor term."""
    n = 2 ** 20
    g = inputs.grid(n, 5.0)
    P = inputs.draw_templates(3, 256, g, precessing=True)
    b = int(np.argmax(P[:, 0] + P[:, 1]))
    idx = np.arange(n - 600, n)
    kw = dict(orbit="kepler", modes=MODES_ALL, precessing=True, gen=20, idx=idx)
    a64, _ = _aet(P[b], g, np.float64, 8, **kw)
    ald, r = _aet(P[b], g, np.longdouble, 8, **kw)
    hp, hc = r.h_grid(idx)
    hmax = max(np.max(np.abs(np.asarray(hp, float))), np.max(np.abs(np.asarray(hc, float))))
    tpl = Template(P[b])
    floor = 32.0 * U64 * n * min(2.0 * (tpl.w_lo + tpl.Delta) * g["dt"], math.pi) * hmax
    scale = np.max(np.abs(ald))
    rel = []
    for c in range(3):
        err = np.max(np.abs(a64[c] - ald[c]))
        rel.append(err / max(np.max(np.abs(ald[c])), scale if c == 2 else 0.0))
        assert err < floor
    assert max(rel) > 1e-9
