"""Fisher matrix by central differences, FP64 (paper Sec. II.C).  Test infrastructure only.

In zero noise at the injection the likelihood Hessian equals the Fisher
matrix Gamma_ij = sum_c (d_i h_c | d_j h_c) (Eq. 2.13), the quantity from
which the paper draws its starting points N(theta_inj, Gamma^-1).  Here the
derivatives are central differences of the ORACLE-M A, E, T series in the
sampler's coordinates.
"""
import numpy as np

from . import likelihood as lk
from .orbits import Orbit
from .response import Response
from .sampler import to_params
from .waveform import Template


def aet(p, g, orbit, taps, modes, precessing, generation):
    r = Response(Template(p), g["t0"], g["dt"], g["n"], Orbit(orbit), taps=taps, modes=modes,
                 precessing=precessing, generation=generation)
    r.cache_full_grid()
    return np.array(r.aet(np.arange(g["n"])))


def fisher(x0, kind, t_c, steps, g, orbit, taps, modes, precessing, generation, channels=(0, 1, 2)):
    x0 = np.asarray(x0, dtype=np.float64)
    d = x0.size
    S = lk.channel_psds(g["n"], g["dt"], generation)
    k_lo, k_hi = lk.band(g["n"], g["dt"], 3e-4, 0.02)
    df = 1.0 / (g["n"] * g["dt"])
    D = []
    for i in range(d):
        xp, xm = x0.copy(), x0.copy()
        xp[i] += steps[i]
        xm[i] -= steps[i]
        hp = aet(to_params(xp, kind, t_c)[0], g, orbit, taps, modes, precessing, generation)
        hm = aet(to_params(xm, kind, t_c)[0], g, orbit, taps, modes, precessing, generation)
        D.append([lk.rfft_dt((hp[c] - hm[c]) / (2.0 * steps[i]), g["dt"]) for c in range(3)])
    G = np.zeros((d, d))
    for i in range(d):
        for j in range(i, d):
            G[i, j] = G[j, i] = sum(lk.inner(D[i][c], D[j][c], S[c], k_lo, k_hi, df) for c in channels)
    return G
