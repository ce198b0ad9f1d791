"""Pins of the oracle's Fourier transform, inner product, PSD and logL (Eqs. 2.12-2.15)."""
import math

import numpy as np
import pytest

from oracle import likelihood as lk
from oracle.orbits import Orbit
from oracle.response import Response
from oracle.waveform import Template
from paper_2501_08261_amd import inputs


@pytest.mark.parametrize("N", [16, 90, 96, 250, 960, 1024, 2160, 4096])
def test_rfft_against_direct_dft(N):
    """P22: numpy rfft (times dt) equals the O(N^2) direct DFT."""
    a = inputs.random_series(N, N)
    got = lk.rfft_dt(a, 5.0)
    want = lk.dft_direct(a, 5.0)
    assert np.max(np.abs(got - want)) < 1e-12 * np.max(np.abs(want))


@pytest.mark.parametrize("N", [1024, 17280])
def test_parseval(N):
    """P21: with S = 1, full band and DC/Nyquist weighted 1/2: (a|a) = 2 dt sum a^2."""
    a = inputs.random_series(7, N)
    dt = 5.0
    af = lk.rfft_dt(a, dt)
    S = np.ones(N // 2 + 1)
    S[0] = S[-1] = 2.0
    got = lk.inner(af, af, S, 0, N // 2, 1.0 / (N * dt))
    assert got == pytest.approx(2 * dt * math.fsum((a * a).tolist()), rel=1e-13)


def test_band_edges():
    """Band of the one-day case: bins 26..1728; the 2^20 case: 1573..104857."""
    assert lk.band(17280, 5.0, 3e-4, 0.02) == (26, 1728)
    assert lk.band(2 ** 20, 5.0, 3e-4, 0.02) == (1573, 104857)


def test_psd_shape():
    f = np.geomspace(1e-4, 0.1, 200)
    Sae, St = lk.psd_sangria(f, "AE"), lk.psd_sangria(f, "T")
    assert np.all(Sae > 0) and np.all(St > 0)
    assert np.all(St[:50] < Sae[:50])              # T is blind at low frequency
    x = 2 * math.pi * f * 2.5e9 / 299792458.0
    assert np.allclose(lk.psd_sangria(f, "AE", 20), Sae * 4 * np.sin(2 * x) ** 2, rtol=1e-14)


def test_loglike_special_cases():
    """P20: logL(h = d) = (d|d)/2 = SNR^2/2, logL_full(h = d) = 0, logL_full <= 0."""
    N, dt = 4096, 5.0
    S = lk.channel_psds(N, dt)
    d = inputs.random_series(1, (3, N), 1e-20)
    h = inputs.random_series(2, (3, N), 1e-20)
    ll, full = lk.loglike(d, d, S, dt)
    assert full == 0.0
    assert ll == pytest.approx(0.5 * lk.noise_inner(d, S, dt), rel=1e-13)
    ll2, full2 = lk.loglike(d, h, S, dt)
    assert full2 < 0
    assert ll2 - full2 == pytest.approx(0.5 * lk.noise_inner(d, S, dt), rel=1e-12)


def test_snr_order_of_magnitude():
    """W1 (weak pin): the one-day M = 1e6 injection at 20 Gpc has an SNR of order 10^3."""
    g, inj, _ = inputs.single_template_case()
    r = Response(Template(inj), g["t0"], g["dt"], g["n"], Orbit("static"), taps=2, modes=((2, 2),))
    r.cache_full_grid()
    aet = np.array(r.aet(np.arange(g["n"])))
    snr = math.sqrt(lk.noise_inner(aet, lk.channel_psds(g["n"], g["dt"]), g["dt"]))
    assert 500 < snr < 20000


def test_colored_noise_matches_its_psd():
    """N3 input: noise drawn from the PSD gives (n|n) = sum of chi-square(2) over the band
    (mean 2 per bin, standard deviation 2 sqrt(bins)), per channel, over several draws."""
    from paper_2501_08261_amd import inputs
    n, dt = 1 << 14, 5.0
    S = lk.channel_psds(n, dt, 20)
    k_lo, k_hi = lk.band(n, dt, 3e-4, 0.02)
    nbins = k_hi - k_lo + 1
    vals = []
    for seed in range(8):
        x = inputs.colored_noise(seed, S, dt)
        for c in range(3):
            xf = lk.rfft_dt(x[c], dt)
            vals.append(lk.inner(xf, xf, S[c], k_lo, k_hi, 1.0 / (n * dt)))
    vals = np.array(vals) / nbins
    assert abs(vals.mean() - 2.0) < 5 * 2.0 / np.sqrt(nbins * len(vals))
    assert abs(vals.std() - 2.0 / np.sqrt(nbins)) < 0.6 * 2.0 / np.sqrt(nbins)


def test_orbit_table_reproduces_kepler():
    """N4: an orbit file sampled every hour from Keplerian ellipses (the input generator's own
    implementation), read by the table orbit's four-point Lagrange interpolation, against the
    oracle's analytic Kepler orbit: positions within the interpolation error bound
    max|r''''| (9/16) h^4 / 4!, where the ellipse's second harmonic (amplitude ~ 3 a e / 2 at
    2 omega) adds 24 e to |r''''| / (a omega^4) = 1 (bound taken with 30 e), plus 1e-4 m of
    rounding on 1.5e11 m coordinates; light times within 1e-11 s."""
    from paper_2501_08261_amd import inputs
    from oracle.phys import AU_SI, YEAR_SI
    h = 3600.0
    tab = inputs.orbit_table(-86400.0, h, 240)
    ot, ok = Orbit("table", table=tab), Orbit("kepler")
    t = np.linspace(0.0, 6e5, 1001)
    om = 2.0 * math.pi / YEAR_SI
    ecc = 2.5e9 / (2.0 * math.sqrt(3.0) * AU_SI)
    bound = AU_SI * om ** 4 * (1.0 + 30.0 * ecc) * (9.0 / 16.0) * h ** 4 / 24.0 + 1e-4
    for k in (1, 2, 3):
        assert np.max(np.abs(ot.position(k, t) - ok.position(k, t))) < bound
    for l in (1, 2, 3, -1, -2, -3):
        assert np.max(np.abs(ot.light_time(l, t) - ok.light_time(l, t))) < 1e-11
    with pytest.raises(ValueError):
        ot.position(1, np.array([-86400.0 + 0.5 * h]))      # before the second sample: not covered
