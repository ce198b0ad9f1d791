"""Pins of the oracle Fisher matrix (P25) and host tests of lt_fisher_draw."""
import ctypes
import math
import os

import numpy as np
import pytest

from oracle import likelihood as olk
from oracle.fisher import fisher, aet
from oracle.sampler import to_params
from paper_2501_08261_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _case():
    g = inputs.grid(2048, 5.0)
    inj = inputs.tab1_injection(False, g, before_end=1000.0)
    x0 = np.array([inj[0], inj[1], inj[4], inj[7], inj[8], inj[9], inj[10], inj[13], inj[12], inj[14]])
    steps = np.array([1.0, 1.0, 1e-4, 1e-4, 1.0, 1e-5, 1e-5, 1e-5, 1e-5, 1e-5])
    return g, inj, x0, steps


def test_fisher_distance_closed_form_and_pd():
    """P25: Gamma_DD = (h|h)/D^2 (h is proportional to 1/D); Gamma symmetric and positive definite."""
    g, inj, x0, steps = _case()
    G = fisher(x0, "aligned10", inj[11], steps, g, "static", 2, ((2, 2), (3, 3)), False, 15)
    h = aet(to_params(x0, "aligned10", inj[11])[0], g, "static", 2, ((2, 2), (3, 3)), False, 15)
    hh = olk.noise_inner(h, olk.channel_psds(g["n"], g["dt"], 15), g["dt"])
    D, eps = x0[4], steps[4]
    # central difference of 1/D: exact factor D^2 / (D^2 - eps^2)^2 * D^2 ... -> (h|h)/D^2 (1 + 2 eps^2/D^2)
    want = hh * D ** 2 / (D ** 2 - eps ** 2) ** 2
    assert G[4, 4] == pytest.approx(want, rel=1e-9)
    assert np.allclose(G, G.T)
    assert np.all(np.linalg.eigvalsh(G / np.sqrt(np.outer(np.diag(G), np.diag(G)))) > -1e-9)


def test_fisher_stable_under_step_halving():
    """P25: central differences converge (Richardson): halving the steps changes Gamma little."""
    g, inj, x0, steps = _case()
    sel = [0, 2, 5, 8]
    G1 = fisher(x0, "aligned10", inj[11], steps, g, "static", 2, ((2, 2),), False, 15)
    G2 = fisher(x0, "aligned10", inj[11], steps / 2, g, "static", 2, ((2, 2),), False, 15)
    for i in sel:
        assert G2[i, i] == pytest.approx(G1[i, i], rel=1e-4)


def test_fisher_draw_covariance():
    """lt_fisher_draw (host code of the library) samples N(x0, Gamma^-1) inside the box."""
    from paper_2501_08261_amd import build
    so = os.path.join(ROOT, "paper_2501_08261_amd", "liblisatd.so")
    if not os.path.exists(so):
        build.build(verbose=False)
    lib = ctypes.CDLL(so)
    f = lib.lt_fisher_draw
    f.argtypes = [ctypes.c_void_p] * 2 + [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                          ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p]
    f.restype = ctypes.c_int
    rng = np.random.default_rng(0)
    d = 4
    A = rng.normal(size=(d, d))
    G = A @ A.T + 0.5 * np.eye(d)
    x0 = np.array([1.0, 2.0, -1.0, 0.5])
    lo, hi = x0 - 100, x0 + 100
    n = 40000
    out = np.zeros((n, d))
    st = f(x0.ctypes.data, G.ctypes.data, d, lo.ctypes.data, hi.ctypes.data, n, 7, 0.0, out.ctypes.data)
    assert st == 0
    C = np.linalg.inv(G)
    assert np.allclose(out.mean(0), x0, atol=4 * np.sqrt(np.diag(C) / n).max())
    assert np.allclose(np.cov(out.T), C, rtol=0.05, atol=0.03 * np.abs(C).max())
    box_lo, box_hi = x0 - 0.5, x0 + 0.5
    st = f(x0.ctypes.data, G.ctypes.data, d, box_lo.ctypes.data, box_hi.ctypes.data, 1000, 7, 0.0, out.ctypes.data)
    assert st == 0 and np.all(out[:1000] >= box_lo) and np.all(out[:1000] <= box_hi)


def test_fisher_draw_badly_scaled():
    """The eigen floor acts in the unit-diagonal basis: a Fisher matrix whose coordinates differ by
    ten decades in scale (masses next to angles) is sampled exactly at reg = 1e-12, where a floor on
    the raw eigenvalues would flatten the large-unit directions."""
    from paper_2501_08261_amd import build
    so = os.path.join(ROOT, "paper_2501_08261_amd", "liblisatd.so")
    if not os.path.exists(so):
        build.build(verbose=False)
    lib = ctypes.CDLL(so)
    f = lib.lt_fisher_draw
    f.argtypes = [ctypes.c_void_p] * 2 + [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                          ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p]
    f.restype = ctypes.c_int
    rng = np.random.default_rng(1)
    d = 4
    A = rng.normal(size=(d, d))
    R = A @ A.T + 0.5 * np.eye(d)
    S = np.diag([1e5, 1.0, 1e-5, 1.0])
    G = S @ R @ S
    w = np.linalg.eigvalsh(G)
    assert w.min() < 1e-12 * w.max()          # a raw-basis floor at 1e-12 would change this matrix
    x0 = np.array([1.0, 2.0, -1.0, 0.5])
    C = np.linalg.inv(G)
    sd = np.sqrt(np.diag(C))
    lo, hi = x0 - 100 * sd, x0 + 100 * sd
    n = 40000
    out = np.zeros((n, d))
    st = f(x0.ctypes.data, G.ctypes.data, d, lo.ctypes.data, hi.ctypes.data, n, 11, 1e-12, out.ctypes.data)
    assert st == 0
    z = (out - x0) / sd
    Cz = C / np.outer(sd, sd)
    assert np.allclose(z.mean(0), 0.0, atol=4 / np.sqrt(n))
    assert np.allclose(np.cov(z.T), Cz, rtol=0.05, atol=0.03)
