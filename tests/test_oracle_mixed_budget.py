"""Error budget of the mixed-precision path, measured on the oracle alone.

The oracle's TDI 2.0 response of the Tab. I precessing injection (Kepler arms, K = 8) is
recomputed with one FP32 rounding planted at a time, and each change is measured in the
noise-weighted norm of the likelihood, |e| / |h|:
* the polarisations stored in FP32 (what the response reads),
* the Lagrange weights of the link responses in FP32 (h at the sender and receiver times),
* the Lagrange weights of the TDI combination in FP32,
* A, E, T stored in FP32.
White roundings (of stored values) stay near FP32's unit roundoff.  Weight roundings do not:
a weight is the same for every output whose delay has the same fraction, so its rounding is a
coherent error, and the TDI 2.0 combination, which cancels the signal to (2 pi f L)^2 of y at
low frequencies, does not cancel it.  In the TDI combination that costs ~3e-5 of |h|: the
reason the response kernel keeps its combined TDI filters, and the sums over them, in FP64.
These measurements back the mixed-precision bounds of the GPU likelihood tests.
"""
import math

import numpy as np

from oracle import likelihood as olk
from oracle import response as ore
from oracle.orbits import Orbit
from oracle.response import Response
from oracle.waveform import Template, MODES_ALL
from paper_2501_08261_amd import inputs


def _f32(x):
    return np.asarray(x).astype(np.float32).astype(np.float64)


def test_mixed_precision_budget(monkeypatch):
    n = 2 ** 14
    g = inputs.grid(n, 5.0)
    S = olk.channel_psds(n, g["dt"], 20)

    def norm(x):
        return math.sqrt(olk.noise_inner(x, S, g["dt"]))

    R = Response(Template(inputs.tab1_injection(True, g)), g["t0"], g["dt"], n, Orbit("kepler"), taps=8,
                 modes=MODES_ALL, precessing=True, generation=20)
    R.cache_full_grid()
    idx = np.arange(n)
    a = np.array(R.aet(idx))
    ha = norm(a)
    rel = {}

    hp, hc = R._hcache
    R._hcache = (_f32(hp), _f32(hc))
    rel["h storage"] = norm(np.array(R.aet(idx)) - a) / ha
    R._hcache = (hp, hc)

    stencil64 = ore._stencil

    def stencil32(s, K):
        nodes, w = stencil64(s, K)
        return nodes, _f32(w)

    y64 = R.y_method

    def y_with(st):
        def y(l, i):
            saved = ore._stencil
            ore._stencil = st
            try:
                return y64(l, i)
            finally:
                ore._stencil = saved
        return y

    monkeypatch.setattr(R, "y_method", y_with(stencil32))
    rel["link weights"] = norm(np.array(R.aet(idx)) - a) / ha
    monkeypatch.setattr(R, "y_method", y_with(stencil64))
    monkeypatch.setattr(ore, "_stencil", stencil32)
    rel["TDI weights"] = norm(np.array(R.aet(idx)) - a) / ha
    monkeypatch.setattr(ore, "_stencil", stencil64)
    rel["A, E, T storage"] = norm(_f32(a) - a) / ha
    print(rel)
    assert rel["h storage"] < 1e-7 and rel["A, E, T storage"] < 1.5e-7
    assert rel["link weights"] < 1e-6
    assert rel["TDI weights"] > 1e-5            # the coherent error a single FP32 filter would carry
    assert sum(v for k, v in rel.items() if k != "TDI weights") < 2e-6
