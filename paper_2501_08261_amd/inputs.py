"""Seeded synthetic workloads shaped like the paper's injections (Tab. I).

This module only draws and lays out input numbers (parameter vectors, grids,
random series).  It holds none of the likelihood arithmetic, so both the HIP
path and the CPU oracle can consume what it produces.

Parameter vector (one FP64 row of 16 per template):
  0 m1 [Msun, detector frame]   1 m2 [Msun]
  2-4 chi1 (x, y, z)            5-7 chi2 (x, y, z)   (L0 frame at f_ref)
  8 D_L [Mpc]  9 iota  10 phi_ref  11 t_c [s, SSB time of the (2,2) peak]
  12 lambda  13 beta  14 psi  15 unused
"""
import math
import numpy as np

N_PARAMS = 16
DEG = math.pi / 180.0


def _spin_cart(a, tilt, phi):
    return [a * math.sin(tilt) * math.cos(phi), a * math.sin(tilt) * math.sin(phi), a * math.cos(tilt)]


def grid(n, dt=5.0, t0=0.0):
    return {"t0": float(t0), "dt": float(dt), "n": int(n)}


def peak_time(g, before_end):
    """SSB time that puts the (2,2) peak `before_end` seconds before the last sample."""
    return g["t0"] + (g["n"] - 1) * g["dt"] - before_end


def tab1_injection(precessing, g, before_end=2000.0):
    """Tab. I injection: m1 = 1e6, m2 = 7e5 Msun, D = 20 Gpc, SNR ~ 2800."""
    p = np.zeros(N_PARAMS)
    p[0], p[1] = 1.0e6, 7.0e5
    if precessing:
        p[2:5] = _spin_cart(0.7, 40.1 * DEG, 40.1 * DEG)
        p[5:8] = _spin_cart(0.4, 22.9 * DEG, 22.9 * DEG)
    else:
        p[4], p[7] = 0.7, 0.4
    p[8] = 2.0e4
    p[9], p[10] = 149.0 * DEG, 229.2 * DEG
    p[11] = peak_time(g, before_end)
    p[12], p[13], p[14] = 34.4 * DEG, -34.4 * DEG, 22.9 * DEG
    return p


def tab1_prior(precessing, inj):
    """Sampling coordinates of the Tab. I injection and the uniform prior box
    (Tab. I ranges; ecliptic latitude restricted to [-pi/2, pi/2]).
    precessing: m1, m2, a1, theta1, phi1, a2, theta2, phi2, D_L[Mpc], iota, phi_ref, beta, lambda, psi;
    aligned: m1, m2, chi1z, chi2z, D_L[Mpc], iota, phi_ref, beta, lambda, psi."""
    tail = [inj[8], inj[9], inj[10], inj[13], inj[12], inj[14]]
    tail_lo = [1.9e4, 0.0, 0.0, -np.pi / 2, 0.0, -np.pi]
    tail_hi = [2.1e4, np.pi, 2 * np.pi, np.pi / 2, 2 * np.pi, np.pi]
    if precessing:
        sp = []
        for c in (2, 5):
            a = float(np.linalg.norm(inj[c:c + 3]))
            sp += [a, float(np.arccos(inj[c + 2] / a)), float(np.arctan2(inj[c + 1], inj[c]))]
        x0 = np.array([inj[0], inj[1]] + sp + tail)
        lo = np.array([0.99e6, 0.69e6, 0.0, 0.0, -np.pi, 0.0, 0.0, -np.pi] + tail_lo)
        hi = np.array([1.01e6, 0.71e6, 1.0, np.pi, np.pi, 1.0, np.pi, np.pi] + tail_hi)
    else:
        x0 = np.array([inj[0], inj[1], inj[4], inj[7]] + tail)
        lo = np.array([0.99e6, 0.69e6, -1.0, -1.0] + tail_lo)
        hi = np.array([1.01e6, 0.71e6, 1.0, 1.0] + tail_hi)
    return x0, lo, hi


def single_template_case():
    """One-day (2,2) case: M = 1e6 Msun, q = 2, chi = (0.5, 0.3), 17,280 samples at 5 s.

    Returns (grid, injection, template offset by 1e-3 in chirp mass at fixed q)."""
    g = grid(17280, 5.0)
    inj = tab1_injection(False, g, before_end=1000.0)
    inj[0], inj[1] = 1.0e6 * 2.0 / 3.0, 1.0e6 / 3.0
    inj[4], inj[7] = 0.5, 0.3
    tmpl = inj.copy()
    tmpl[0] *= 1.001
    tmpl[1] *= 1.001
    return g, inj, tmpl


def draw_templates(seed, batch, g, precessing, before_end=2000.0):
    """Random templates: log10 M ~ U[5, 7], q ~ U[1, 10], isotropic sky / orientation.

    Aligned: chi_z ~ U[-0.99, 0.99].  Precessing: |chi| ~ U[0, 0.99] with
    isotropic directions.  D = 20 Gpc; (2,2) peak `before_end` s before the end.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    p = np.zeros((batch, N_PARAMS))
    M = 10.0 ** rng.uniform(5.0, 7.0, batch)
    q = rng.uniform(1.0, 10.0, batch)
    p[:, 0], p[:, 1] = M * q / (1.0 + q), M / (1.0 + q)
    if precessing:
        for j, col in ((0, 2), (1, 5)):
            a = rng.uniform(0.0, 0.99, batch)
            ct = rng.uniform(-1.0, 1.0, batch)
            ph = rng.uniform(0.0, 2.0 * math.pi, batch)
            st = np.sqrt(1.0 - ct * ct)
            p[:, col], p[:, col + 1], p[:, col + 2] = a * st * np.cos(ph), a * st * np.sin(ph), a * ct
    else:
        p[:, 4] = rng.uniform(-0.99, 0.99, batch)
        p[:, 7] = rng.uniform(-0.99, 0.99, batch)
    p[:, 8] = 2.0e4
    p[:, 9] = np.arccos(rng.uniform(-1.0, 1.0, batch))
    p[:, 10] = rng.uniform(0.0, 2.0 * math.pi, batch)
    p[:, 11] = peak_time(g, before_end)
    p[:, 12] = rng.uniform(0.0, 2.0 * math.pi, batch)
    p[:, 13] = np.arcsin(rng.uniform(-1.0, 1.0, batch))
    p[:, 14] = rng.uniform(0.0, math.pi, batch)
    return p


def random_series(seed, shape, scale=1.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    return scale * rng.standard_normal(shape)


def colored_noise(seed, S, dt):
    """Stationary Gaussian noise [3][n] with one-sided PSDs S [3][n/2+1] (bin 0 ignored).

    Drawn in the frequency domain with E|n~_k|^2 = S_k / (2 df), n~ = dt * DFT(n), df = 1/(n dt):
    real and imaginary parts N(0, S_k / (4 df)) for 0 < k < n/2, a real Nyquist bin of
    variance S / (2 df), no DC; then n = inverse real DFT of n~ / dt.  With the inner product
    (a|b) = 4 df Re sum a~ conj(b~) / S, each band bin adds a chi-square with two degrees of
    freedom to (n|n): mean 2 per bin."""
    S = np.asarray(S, dtype=np.float64)
    nb = S.shape[-1]
    n = 2 * (nb - 1)
    df = 1.0 / (n * dt)
    rng = np.random.Generator(np.random.PCG64(seed))
    re = rng.standard_normal((3, nb))
    im = rng.standard_normal((3, nb))
    sig = np.zeros_like(S)
    sig[:, 1:] = np.sqrt(S[:, 1:] / (4.0 * df))
    nf = sig * (re + 1j * im)
    nf[:, 0] = 0.0
    nf[:, -1] = np.sqrt(2.0) * sig[:, -1] * re[:, -1]
    return np.fft.irfft(nf / dt, n=n, axis=-1)


# synthetic orbit files: published constants (c by definition, the IAU astronomical unit,
# one sidereal year) and the nominal LISA arm
_C, _AU, _YEAR, _ARM = 299792458.0, 1.495978707e11, 31558149.763545603, 2.5e9


def orbit_table(t0, dt, n, arm=_ARM, au=_AU, phase0=0.0, t_ref=0.0):
    """A synthetic orbit file on the times t0 + j dt, j < n, in the layout of
    lt_orbit's table kind: positions [n][3][3] (spacecraft 1..3, x y z in m) and light
    times [n][6] (links 1, 2, 3, -1, -2, -3, for reception at each time).

    The spacecraft fly first-order "cartwheel" Keplerian ellipses around the Sun
    (semi-major axis au, eccentricity arm / (2 sqrt(3) au), inclination sqrt(3) times
    the eccentricity, mean anomalies and perihelion longitudes 2 pi / 3 apart); Kepler's
    equation is solved by Newton's method, and each light time L by iterating
    L = |r_receiver(t) - r_sender(t - L)| / c.  Link l: sender (|l| + 1) mod 3 + 1 and
    receiver |l| mod 3 + 1 for l > 0, swapped for l < 0.
    Returns (t0, dt, pos, ltt)."""
    t = t0 + dt * np.arange(n, dtype=np.float64)
    e = arm / (2.0 * math.sqrt(3.0) * au)
    inc = math.sqrt(3.0) * e

    def pos(k, tt):
        sig = 2.0 * math.pi * (k - 1) / 3.0
        M = 2.0 * math.pi / _YEAR * (tt - t_ref) + phase0 - sig
        E = M.copy()
        for _ in range(60):
            E = E - (E - e * np.sin(E) - M) / (1.0 - e * np.cos(E))
        xo = au * (np.cos(E) - e)
        yo = au * math.sqrt(1.0 - e * e) * np.sin(E)
        x1, z1 = xo * math.cos(inc), xo * math.sin(inc)
        return np.stack([math.cos(sig) * x1 - math.sin(sig) * yo, math.sin(sig) * x1 + math.cos(sig) * yo, z1], -1)

    P = np.stack([pos(k, t) for k in (1, 2, 3)], 1)                 # [n][3][3]
    L = np.zeros((n, 6))
    for c, l in enumerate((1, 2, 3, -1, -2, -3)):
        a = abs(l)
        s, r = (a + 1) % 3 + 1, a % 3 + 1
        if l < 0:
            s, r = r, s
        rr = P[:, r - 1]
        Ll = np.linalg.norm(rr - P[:, s - 1], axis=-1) / _C
        for _ in range(30):
            Ll = np.linalg.norm(rr - pos(s, t - Ll), axis=-1) / _C
        L[:, c] = Ll
    return t0, dt, P, L
