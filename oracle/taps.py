"""Choice of the interpolation order K at delayed times (paper Sec. II.B interpolates linearly;
the order is a parameter of the method here).  Test infrastructure only.

The interpolation error of the method is ORACLE-M(K) - ORACLE-X (response.py): A, E, T with
h and y interpolated by K-tap Lagrange against A, E, T with h evaluated at every exact delayed
time.  It is measured away from the grid's edges (where ORACLE-M reads zeros outside the grid
and ORACLE-X does not) in the metric of the parity tests: max |M - X| over the samples and
channels, relative to max |X|.  The chosen K is the smallest one whose error stays below a
stated tolerance for every template of a set; larger K cost more work and buy no accuracy
once the error is below the rounding floor of the arithmetic that follows.
"""
import numpy as np

from .orbits import Orbit
from .response import Response
from .waveform import Template, MODES_ALL


def interp_error(p, K, g, idx, orbit="kepler", generation=20, modes=MODES_ALL, precessing=True):
    """max |ORACLE-M(K) - ORACLE-X| / max |ORACLE-X| of A, E, T at grid indices idx."""
    x = np.array(Response(Template(p), g["t0"], g["dt"], g["n"], Orbit(orbit), taps=2, modes=modes,
                          precessing=precessing, generation=generation).aet(idx, exact=True))
    r = Response(Template(p), g["t0"], g["dt"], g["n"], Orbit(orbit), taps=K, modes=modes, precessing=precessing,
                 generation=generation)
    r.cache_full_grid()
    m = np.array(r.aet(idx))
    return float(np.max(np.abs(m - x)) / np.max(np.abs(x)))


def choose_taps(params, g, idx, tol, candidates=(2, 4, 6, 8, 12, 16, 24, 32), **kw):
    """Smallest K of `candidates` whose interp_error is below tol for every template in params;
    returns (K, {K: worst error}) with the errors of the candidates tried (None: none passes)."""
    worst = {}
    for K in candidates:
        worst[K] = max(interp_error(p, K, g, idx, **kw) for p in params)
        if worst[K] < tol:
            return K, worst
    return None, worst
