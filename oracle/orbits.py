"""Spacecraft orbits and light travel times, FP64 (paper Sec. II.B).  Test infrastructure only.

The paper takes positions and light travel times from the LDC AnalyticOrbit
class (equal arms) and ESA orbit files (unequal arms); neither is printed, so
two analytic orbit kinds are defined here (reading of the orbit input):

* "static": an exact equilateral triangle of side L, centroid at (1 AU, 0, 0),
  plane inclined 60 degrees to the ecliptic (normal tilted towards the Sun);
  every light travel time is exactly L / c.
* "table": positions and light travel times sampled on a uniform time grid
  (an orbit file), interpolated with four-point Lagrange weights on the
  samples j-1 .. j+2 around t; receiver at t, sender at t - L(t).
* "kepler": three exact heliocentric Keplerian ellipses with semi-major axis
  1 AU, eccentricity e = L / (2 sqrt(3) AU) and inclination sqrt(3) e (the
  first-order "cartwheel" parameters), perihelion longitudes and mean
  anomalies offset by 2 pi / 3.  Kepler's equation is solved by Newton
  iteration and the light travel time of each link from the implicit
  equation L = |r_r(t) - r_s(t - L)| / c by fixed-point iteration.  The arms
  breathe at O(e^2), so the six light times differ and vary in time.

Agreement with LDC / ESA orbits is parity unpinned.
"""
import math
import numpy as np

from .phys import AU_SI, C_SI, YEAR_SI, ARM_SI

# link label l -> (sender, receiver); positive l: 1: 3->2, 2: 1->3, 3: 2->1
LINK_LABELS = (1, 2, 3, -1, -2, -3)


def link_ends(l):
    k = abs(l)
    s, r = (k + 1) % 3 + 1, k % 3 + 1
    return (s, r) if l > 0 else (r, s)


def _table_interp(t, t0, dt, v):
    """Four-point Lagrange interpolation of rows v[j] (time t0 + j dt) at times t: [len(t), ...]."""
    x = (np.asarray(t, dtype=np.float64) - t0) / dt
    j = np.floor(x)
    if np.any(j < 1) or np.any(j + 2 > len(v) - 1):
        raise ValueError("orbit table does not cover the requested times")
    f = x - j
    j = j.astype(np.int64)
    w = [-f * (f - 1) * (f - 2) / 6.0, (f + 1) * (f - 1) * (f - 2) / 2.0, -(f + 1) * f * (f - 2) / 2.0,
         (f + 1) * f * (f - 1) / 6.0]
    out = 0.0
    for m in range(4):
        wm = w[m].reshape(w[m].shape + (1,) * (v.ndim - 1))
        out = out + wm * v[j - 1 + m]
    return out


class Orbit:
    def __init__(self, kind="static", arm=ARM_SI, au=AU_SI, phase0=0.0, t_ref=0.0, table=None):
        if kind not in ("static", "kepler", "table"):
            raise ValueError(kind)
        self.kind, self.arm, self.au, self.phase0, self.t_ref = kind, arm, au, phase0, t_ref
        if kind == "table":
            self.tab_t0, self.tab_dt, pos, ltt = table
            self.tab_pos = np.asarray(pos, dtype=np.float64)
            self.tab_ltt = np.asarray(ltt, dtype=np.float64)
        self.ecc = arm / (2.0 * math.sqrt(3.0) * au)
        self.incl = math.sqrt(3.0) * self.ecc
        self.Omega = 2.0 * math.pi / YEAR_SI

    def position(self, k, t):
        """Position [3, len(t)] of spacecraft k (1..3) at times t [s]."""
        t = np.atleast_1d(np.asarray(t, dtype=np.float64))
        if self.kind == "table":
            return _table_interp(t, self.tab_t0, self.tab_dt, self.tab_pos[:, k - 1, :]).T
        sig = 2.0 * math.pi * (k - 1) / 3.0
        if self.kind == "static":
            rho = self.arm / math.sqrt(3.0)
            e1 = np.array([0.5, 0.0, math.sqrt(3.0) / 2.0])
            e2 = np.array([0.0, 1.0, 0.0])
            p = np.array([self.au, 0.0, 0.0]) + rho * (math.cos(sig) * e1 + math.sin(sig) * e2)
            return np.repeat(p[:, None], t.size, axis=1)
        e, a = self.ecc, self.au
        Mk = self.Omega * (t - self.t_ref) + self.phase0 - sig
        E = Mk.copy()
        for _ in range(50):
            dE = (E - e * np.sin(E) - Mk) / (1.0 - e * np.cos(E))
            E = E - dE
            if np.max(np.abs(dE)) < 1e-17:
                break
        xo = a * (np.cos(E) - e)
        yo = a * math.sqrt(1.0 - e * e) * np.sin(E)
        x1, z1 = xo * math.cos(self.incl), xo * math.sin(self.incl)
        cs, ss = math.cos(sig), math.sin(sig)
        return np.stack([cs * x1 - ss * yo, ss * x1 + cs * yo, z1])

    def light_time(self, l, t):
        """Light travel time [s] of link l for reception time t."""
        t = np.atleast_1d(np.asarray(t, dtype=np.float64))
        if self.kind == "table":
            return _table_interp(t, self.tab_t0, self.tab_dt, self.tab_ltt[:, LINK_LABELS.index(l)])
        if self.kind == "static":
            return np.full(t.shape, self.arm / C_SI)
        s, r = link_ends(l)
        rr = self.position(r, t)
        L = np.linalg.norm(rr - self.position(s, t), axis=0) / C_SI
        for _ in range(20):
            Ln = np.linalg.norm(rr - self.position(s, t - L), axis=0) / C_SI
            done = np.max(np.abs(Ln - L)) < 1e-15
            L = Ln
            if done:
                break
        return L
