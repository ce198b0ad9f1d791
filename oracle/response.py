"""LISA link responses, TDI and A, E, T, FP64 (paper Sec. II.B, Eqs. 2.7-2.11).

Test infrastructure only.  Two levels:

* ORACLE-M ("method"): h+, hx on the uniform grid, link responses y_slr on
  the grid with h interpolated at the delayed times by centred K-tap Lagrange
  interpolation, TDI from y interpolated the same way.  This is the parity
  target of the GPU path (same K).
* ORACLE-X ("exact"): no interpolation at all; h is evaluated analytically at
  every exact delayed time and y directly at every exact TDI delay.
  ORACLE-X minus ORACLE-M is the interpolation error of the method.

Readings (listed in the design notes):
* Eq. (2.8): y = [x+ (h+(t_s) - h+(t_r)) + xx (hx(t_s) - hx(t_r))] / (1 - k.n)
  with x+ = ((u.n)^2 - (v.n)^2) / 2 and xx = (u.n)(v.n), i.e. the projection
  n.h.n / 2 of h = h+ (uu - vv) + hx (uv + vu); the receiver position is taken
  at the reception time t, the sender position at the emission time t - L_l(t),
  t_s = t - L_l(t) - k.r_s / c and t_r = t - k.r_r / c.
* Eq. (2.10), eleventh term: the delay is read as 2L_-2 + L_2 + 2L_3 + 2L_-3
  (the printed one cancels the twelfth term).
* Every TDI delay is a plain sum of light times evaluated at the reception
  time t of the TDI sample.
* Interpolation: nodes j0 - K/2 + 1 .. j0 + K/2 with j0 = floor((tau - t0)/dt);
  samples outside [0, N) read as zero; K = 2 is linear interpolation.
"""
import math
import numpy as np

from .phys import C_SI
from .orbits import link_ends
from .twist import polarizations
from .waveform import MODES_ALL, real_array


def k_u_v(lam, beta):
    """Propagation direction and polarisation vectors, Eq. (2.7)."""
    cl, sl, cb, sb = math.cos(lam), math.sin(lam), math.cos(beta), math.sin(beta)
    k = np.array([-cb * cl, -cb * sl, -sb])
    v = np.array([-sb * cl, -sb * sl, cb])
    u = np.array([sl, -cl, 0.0])
    return k, u, v


def lagrange_offsets(K):
    return np.arange(-K // 2 + 1, K // 2 + 1)


def lagrange_weights(frac, K):
    """w_i(frac) = prod_{j != i} (frac - o_j) / (o_i - o_j), offsets o = -K/2+1..K/2."""
    o = lagrange_offsets(K)
    frac = real_array(frac)
    w = np.ones(frac.shape + (K,), dtype=frac.dtype)
    for i in range(K):
        for j in range(K):
            if j != i:
                w[..., i] *= (frac - o[j]) / (o[i] - o[j])
    return w


def _stencil(s, K):
    """Nodes [.., K] and Lagrange weights [.., K] for fractional grid index s."""
    j0 = np.floor(s).astype(np.int64)
    return j0[..., None] + lagrange_offsets(K), lagrange_weights(s - j0, K)


def _lookup(values, uniq, nodes, N):
    """Values at grid `nodes` from (uniq, values) tables; zero outside [0, N)."""
    valid = (nodes >= 0) & (nodes < N)
    out = np.zeros(nodes.shape)
    out[valid] = values[np.searchsorted(uniq, nodes[valid])]
    return out


def _needed(node_arrays, N):
    allnodes = np.concatenate([a.ravel() for a in node_arrays])
    return np.unique(allnodes[(allnodes >= 0) & (allnodes < N)])


# TDI term lists: (sign, link label, [delay link labels]) -- Eqs. (2.9), (2.10)
X15 = ((+1, -3, (3, 2, -2)), (-1, -3, (3,)), (+1, 3, (2, -2)), (-1, 3, ()),
       (+1, 2, (-2,)), (-1, 2, (-2, -3, 3)), (+1, -2, ()), (-1, -2, (-3, 3)))
X20 = X15[:2] + ((+1, -3, (-2, 2, 3, 3, -3)), (-1, -3, (3, 3, -3, -2, -2, 2, 2))) \
    + X15[2:4] + ((+1, 3, (-2, 2, 3, -3)), (-1, 3, (3, -3, -2, -2, 2, 2))) \
    + X15[4:6] + ((+1, 2, (-2, -2, 2, 3, 3, -3, -3)), (-1, 2, (3, -3, -2, -2, 2))) \
    + X15[6:8] + ((+1, -2, (-2, 2, 3, 3, -3, -3)), (-1, -2, (3, -3, -2, 2)))


def cyclic(l, times):
    """Relabel link l under spacecraft permutation 1->2->3->1 applied `times` times."""
    s = 1 if l > 0 else -1
    k = abs(l)
    for _ in range(times):
        k = k % 3 + 1
    return s * k


def tdi_terms(generation, channel):
    base = X15 if generation == 15 else X20
    return tuple((sg, cyclic(l, channel), tuple(cyclic(d, channel) for d in dl)) for sg, l, dl in base)


class Response:
    """One template on one grid with one orbit (hot-path steps a4-a8)."""

    def __init__(self, tpl, t0, dt, N, orbit, taps=2, modes=MODES_ALL, precessing=False,
                 generation=15, hfun=None, sky=None, coarse=1, real=np.float64):
        """hfun: optional callable t -> (h+, hx) replacing the waveform (used by
        the plane-wave checks); sky: optional (lambda, beta) overriding tpl's;
        coarse = 2: the polarisations on the grid are the waveform on every second
        sample (even indices) and the mean of the two neighbours on the others
        (linear interpolation from a grid of twice the step, Sec. II.C); real:
        np.float64, or np.longdouble for the sample and delayed times of the
        extended-precision reference (with a Template of the same precision)."""
        self.real = real
        self.coarse = int(coarse)
        self.tpl, self.t0, self.dt, self.N = tpl, float(t0), float(dt), int(N)
        self.hfun = hfun
        self.orbit, self.K, self.modes = orbit, int(taps), modes
        self.precessing, self.generation = precessing, generation
        lam, bet = sky if sky is not None else (tpl.lam, tpl.beta)
        self.k, self.u, self.v = k_u_v(lam, bet)
        self._hcache = None

    # -- polarisations ------------------------------------------------------
    def _times(self, idx):
        """Sample times t0 + idx dt in the response's precision."""
        if self.real is np.float64:
            return self.t0 + idx * self.dt
        return self.real(self.t0) + np.asarray(idx).astype(self.real) * self.real(self.dt)

    def h_exact(self, t):
        if self.hfun is not None:
            return self.hfun(real_array(t))
        return polarizations(self.tpl, real_array(t), self.modes, self.precessing)

    def h_grid(self, idx):
        idx = np.asarray(idx, dtype=np.int64)
        if self._hcache is not None:
            return self._hcache[0][idx], self._hcache[1][idx]
        if self.coarse == 2:
            lo = idx - (idx % 2)
            a = self.h_exact(self._times(lo))
            b = self.h_exact(self._times(lo + 2))
            odd = (idx % 2) == 1
            return tuple(np.where(odd, 0.5 * (a[q] + b[q]), a[q]) for q in range(2))
        return self.h_exact(self._times(idx))

    def cache_full_grid(self):
        if self.coarse == 2:
            self._hcache = None
            hp, hc = self.h_grid(np.arange(self.N))
            self._hcache = (hp, hc)
            return
        hp, hc = self.h_exact(self._times(np.arange(self.N)))
        self._hcache = (hp, hc)

    # -- one link -----------------------------------------------------------
    def link_geometry(self, l, tau):
        """x+/(1-k.n), xx/(1-k.n), t_s, t_r for link l at reception times tau."""
        s, r = link_ends(l)
        L = self.orbit.light_time(l, tau)
        rr = self.orbit.position(r, tau)
        rs = self.orbit.position(s, tau - L)
        d = rr - rs
        n = d / np.linalg.norm(d, axis=0)
        un, vn, kn = self.u @ n, self.v @ n, self.k @ n
        pp = 0.5 * (un * un - vn * vn) / (1.0 - kn)
        pc = un * vn / (1.0 - kn)
        t_s = tau - L - (self.k @ rs) / C_SI
        t_r = tau - (self.k @ rr) / C_SI
        return pp, pc, t_s, t_r

    def y_method(self, l, idx):
        """ORACLE-M link response y_l on grid indices idx (h interpolated)."""
        idx = np.asarray(idx, dtype=np.int64)
        tau = self._times(idx)
        pp, pc, t_s, t_r = self.link_geometry(l, tau)
        ns, ws = _stencil((t_s - self.t0) / self.dt, self.K)
        nr, wr = _stencil((t_r - self.t0) / self.dt, self.K)
        need = _needed([ns, nr], self.N)
        hp, hc = self.h_grid(need) if need.size else (np.zeros(0), np.zeros(0))
        dhp = np.sum(ws * _lookup(hp, need, ns, self.N), -1) - np.sum(wr * _lookup(hp, need, nr, self.N), -1)
        dhc = np.sum(ws * _lookup(hc, need, ns, self.N), -1) - np.sum(wr * _lookup(hc, need, nr, self.N), -1)
        return pp * dhp + pc * dhc

    def y_exact(self, l, tau):
        """ORACLE-X link response at arbitrary reception times (no interpolation)."""
        pp, pc, t_s, t_r = self.link_geometry(l, real_array(tau))
        hs, hr = self.h_exact(t_s), self.h_exact(t_r)
        return pp * (hs[0] - hr[0]) + pc * (hs[1] - hr[1])

    # -- TDI ----------------------------------------------------------------
    def xyz(self, idx, exact=False):
        """X, Y, Z at output grid indices idx (ORACLE-M, or ORACLE-X if exact)."""
        idx = np.asarray(idx, dtype=np.int64)
        t = self._times(idx)
        Lt = {l: self.orbit.light_time(l, t) for l in (1, 2, 3, -1, -2, -3)}
        terms = []
        for ch in range(3):
            for sg, l, dl in tdi_terms(self.generation, ch):
                D = np.zeros(t.shape)
                for d in dl:
                    D = D + Lt[d]
                terms.append((ch, sg, l, t - D))
        out = [np.zeros(t.shape) for _ in range(3)]
        if exact:
            for ch, sg, l, tau in terms:
                out[ch] = out[ch] + sg * self.y_exact(l, tau)
            return out
        stencils = [(ch, sg, l) + _stencil((tau - self.t0) / self.dt, self.K) for ch, sg, l, tau in terms]
        ytab = {}
        for l in (1, 2, 3, -1, -2, -3):
            need = _needed([n for _, _, ll, n, _ in stencils if ll == l], self.N)
            ytab[l] = (need, self.y_method(l, need) if need.size else np.zeros(0))
        for ch, sg, l, nodes, w in stencils:
            need, yv = ytab[l]
            out[ch] = out[ch] + sg * np.sum(w * _lookup(yv, need, nodes, self.N), -1)
        return out

    def aet(self, idx, exact=False):
        """A, E, T of Eq. (2.11) at output grid indices idx."""
        X, Y, Z = self.xyz(idx, exact)
        return (Z - X) / math.sqrt(2.0), (X - 2.0 * Y + Z) / math.sqrt(6.0), (X + Y + Z) / math.sqrt(3.0)
