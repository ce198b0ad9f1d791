"""PSD, Fourier transform, inner products and log-likelihood, FP64 (paper Sec. II.B).

Test infrastructure only.  Readings (listed in the design notes):

* Eq. (2.13) discretised: a~_k = dt sum_n a_n exp(-2 pi i k n / N),
  f_k = k / (N dt), (a|b) = 4 df Re sum_{k=k_lo}^{k_hi} a~_k conj(b~_k) / S(f_k),
  df = 1/(N dt); the band is every bin with f_lo <= f_k <= f_hi (bin edges
  taken with a relative slack of 1e-12 so that f_hi = 0.02 Hz on a one-day
  5 s grid keeps bin 1728); no window, no padding.
* Eq. (2.12) is read with the sign of its footnote:
  logL = sum_c [(d_c|h_c) - (h_c|h_c)/2] and logL_full = -1/2 sum_c (h_c-d_c|h_c-d_c).
* Eqs. (2.14)-(2.15): the printed trigonometric arguments are read with
  x = 2 pi f L / c; the acceleration amplitude is 2.4e-15 m s^-2 Hz^-1/2; for
  TDI 2.0 the PSDs gain the factor 4 sin^2(2x).
"""
import math
import numpy as np

from .phys import C_SI, ARM_SI

BAND_SLACK = 1e-12


def psd_sangria(f, channel, generation=15, arm=ARM_SI, s_acc=2.4e-15, s_oms=7.9e-12):
    """One-sided PSD of channel 'AE' or 'T' at frequencies f (f > 0)."""
    f = np.asarray(f, dtype=np.float64)
    x = 2.0 * math.pi * f * arm / C_SI
    w = 2.0 * math.pi * f / C_SI
    Sacc = s_acc ** 2 * (1.0 + (4e-4 / f) ** 2) * (1.0 + (f / 8e-3) ** 4) * (2.0 * math.pi * f) ** -4 * w ** 2
    Sop = s_oms ** 2 * (1.0 + (2e-3 / f) ** 4) * w ** 2
    s2 = np.sin(x) ** 2
    if channel == "AE":
        S = 8.0 * s2 * (2.0 * Sacc * (3.0 + 2.0 * np.cos(x) + np.cos(2.0 * x)) + Sop * (2.0 + np.cos(x)))
    elif channel == "T":
        S = 16.0 * Sop * (1.0 - np.cos(x)) * s2 + 128.0 * Sacc * s2 * np.sin(0.5 * x) ** 4
    else:
        raise ValueError(channel)
    if generation == 20:
        S = S * 4.0 * np.sin(2.0 * x) ** 2
    return S


def band(N, dt, f_lo, f_hi):
    """Inclusive bin range [k_lo, k_hi] of the likelihood band."""
    T = N * dt
    k_lo = math.ceil(f_lo * T * (1.0 - BAND_SLACK))
    k_hi = math.floor(f_hi * T * (1.0 + BAND_SLACK))
    return max(k_lo, 0), min(k_hi, N // 2)


def rfft_dt(a, dt):
    """Continuous-FT approximation a~_k = dt * DFT(a)_k, k = 0..N/2 (numpy pocketfft)."""
    return np.fft.rfft(np.asarray(a, dtype=np.float64)) * dt


def dft_direct(a, dt):
    """O(N^2) direct DFT, for pinning rfft_dt on small N."""
    a = np.asarray(a, dtype=np.float64)
    N = a.size
    n = np.arange(N)
    k = np.arange(N // 2 + 1)
    return dt * np.exp(-2j * math.pi * np.outer(k, n) / N) @ a


def inner(af, bf, S, k_lo, k_hi, df):
    """(a|b) = 4 df Re sum_k a~ conj(b~) / S over the band (math.fsum)."""
    sl = slice(k_lo, k_hi + 1)
    terms = (np.asarray(af)[sl] * np.conj(np.asarray(bf)[sl])).real / np.asarray(S)[sl]
    return 4.0 * df * math.fsum(terms.tolist())


def channel_psds(N, dt, generation=15, arm=ARM_SI):
    """PSD arrays [3][N/2+1] for A, E, T on the rfft grid (bin 0 set to +inf)."""
    f = np.arange(N // 2 + 1) / (N * dt)
    out = np.full((3, f.size), np.inf)
    out[0, 1:] = psd_sangria(f[1:], "AE", generation, arm)
    out[1, 1:] = out[0, 1:]
    out[2, 1:] = psd_sangria(f[1:], "T", generation, arm)
    return out


def loglike(d_aet, h_aet, S, dt, f_lo=3e-4, f_hi=0.02):
    """(logL, logL_full) of Eq. (2.12) as read above; d_aet, h_aet are [3][N] time series."""
    d_aet, h_aet = np.asarray(d_aet), np.asarray(h_aet)
    N = d_aet.shape[-1]
    df = 1.0 / (N * dt)
    k_lo, k_hi = band(N, dt, f_lo, f_hi)
    logl_terms, full_terms = [], []
    for c in range(3):
        df_, hf_ = rfft_dt(d_aet[c], dt), rfft_dt(h_aet[c], dt)
        dh = inner(df_, hf_, S[c], k_lo, k_hi, df)
        hh = inner(hf_, hf_, S[c], k_lo, k_hi, df)
        rf = rfft_dt(h_aet[c] - d_aet[c], dt)
        rr = inner(rf, rf, S[c], k_lo, k_hi, df)
        logl_terms += [dh, -0.5 * hh]
        full_terms.append(-0.5 * rr)
    return math.fsum(logl_terms), math.fsum(full_terms)


def noise_inner(x_aet, S, dt, f_lo=3e-4, f_hi=0.02):
    """sum_c (x_c|x_c) over the band."""
    x_aet = np.asarray(x_aet)
    N = x_aet.shape[-1]
    k_lo, k_hi = band(N, dt, f_lo, f_hi)
    tot = []
    for c in range(3):
        xf = rfft_dt(x_aet[c], dt)
        tot.append(inner(xf, xf, S[c], k_lo, k_hi, 1.0 / (N * dt)))
    return math.fsum(tot)
