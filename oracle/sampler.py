"""Parallel-tempered ensemble MCMC in numpy (paper Sec. II.C).  Test infrastructure only.

The paper drives its likelihood with ptemcee (parallel-tempered affine-
invariant ensemble sampler) from Fisher-initialised walkers; its settings are
not printed.  This oracle fixes one reading and is the step-by-step reference
of the GPU sampler:

* Goodman-Weare stretch move on the two halves of each temperature's
  ensemble: for walker k of half h, partner j uniform in the other half,
  z = ((a - 1) u + 1)^2 / a (density ~ 1/sqrt(z) on [1/a, a]),
  Y = X_j + z (X_k - X_j), accepted when
  ln u' < (d - 1) ln z + beta (logL_Y - logL_X) + (logP_Y - logP_X);
* uniform-box prior (Tab. I ranges);
* after both halves, adjacent-temperature swaps from the hottest pair down:
  walker k at beta_i against walker (k + r) mod W at beta_{i+1}, accepted with
  min(1, exp((beta_i - beta_{i+1}) (logL_{i+1} - logL_i)));
* geometric ladder beta_i = t_max^(-i / (T - 1));
* optional learned-proposal move (a normalising flow q, see oracle.flow):
  after both halves and before the swaps, every walker of the coldest rung
  proposes y = flow inverse of z, z standard normal from Box-Muller pairs
  (Philox counter (step, 0x400, walker, q) -> coordinates 4q..4q+3), accepted
  when ln u < beta_0 (logL_y - logL_x) + (logP_y - logP_x) + ln q(x) - ln q(y)
  (independence Metropolis-Hastings), u from counter (step, 0x500, walker, 0);
* optional symmetry fold of that move, for a target invariant under
  x_i -> x_i + P (the polarisation angle, P = pi: h carries exp(2 i psi)):
  the flow sees x_i folded into [c, c + P); a flow sample y_f with its i-th
  coordinate in that window becomes the copy y_i = y_f,i + (k_min + j) P,
  j = floor(u n) of the n copies inside [lo_i, hi_i], u from counter
  (step, 0x600, walker, 0), and both ln q carry - ln n (the proposal density
  of a copy is q_flow(y_f) / n), so the ratio stays exact; a y_f outside the
  window is outside the proposal's range and is rejected;
* mixture with the plain move (the learned proposal mixed with the stretch move at rate
  p_flow): each step runs the flow move only when u < p_flow, u from counter
  (step, 0x800, 0, 0); a step without it proposes nothing for it.  Every step's kernel
  (stretch move, flow move, swaps) keeps the target, and the choice does not depend on the
  state, so the mixture keeps it too; p_flow = 1 runs the flow move every step;
  optionally (exclusive) a step that runs the flow move skips the stretch move on the
  cold rung (its rows are neither proposed nor counted): the cold rung's kernel on that
  step is then the flow move alone, again a state-independent choice between kernels
  that keep the target;
* optional mixture of two flows (one per mode of a two-mode posterior): the proposal
  density is q = w1 q1 + (1 - w1) q2.  Each walker draws its component, flow 1 when
  u < w1 with u from counter (step, 0x900, walker, 0); both flows map the same base
  normals, and the walker takes its component's point.  log q of the proposal and of
  the current (folded) position is the mixture's, log(w1 q1 + w2 q2) from both flows'
  forward passes, so the independence acceptance above is the exact one for q;
* optional latent random walk in place of the independence proposal:
  z = f(x) (the flow's forward map of the folded position), z' = z + w eps,
  eps standard normal from counter (step, 0x700, walker, q) like the base
  samples, y = f^-1(z'); the walk is symmetric in z, so q(x) and q(y) above
  become q(x) / N(z) and q(y) / N(z') (the Jacobians of f), with
  ln N(z) = -|z|^2 / 2 - (d / 2) ln 2 pi summed in coordinate order;
* random numbers from Philox4x32-10 (Salmon, Moraes, Dror, Shaw 2011) keyed
  by the seed, counter (step, purpose, slot, 0), uniforms (u + 1/2) 2^-32.
"""
import math

import numpy as np

from . import flow as _flow

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF
TAG_MOVE, TAG_SHIFT, TAG_SWAP, TAG_FLOWZ, TAG_FLOWU, TAG_FLOWC, TAG_FLOWW = (0x100, 0x200, 0x300, 0x400, 0x500,
                                                                     0x600, 0x700)
TAG_FLOWG = 0x800
TAG_FLOWM = 0x900


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds on arrays of counters [..., 4] and a key (k0, k1)."""
    c = [np.asarray(ctr[..., i], dtype=np.uint64) for i in range(4)]
    k0, k1 = np.uint64(key[0]), np.uint64(key[1])
    m0, m1 = np.uint64(M0), np.uint64(M1)
    mask = np.uint64(MASK)
    for r in range(10):
        if r > 0:
            k0 = (k0 + np.uint64(W0)) & mask
            k1 = (k1 + np.uint64(W1)) & mask
        p0 = m0 * c[0]
        p1 = m1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & mask
        hi1, lo1 = p1 >> np.uint64(32), p1 & mask
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return np.stack(c, axis=-1).astype(np.uint64)


def u01(u):
    return (np.asarray(u, dtype=np.float64) + 0.5) * 2.0 ** -32


def _ctr(step, tag, slots, lane=0):
    slots = np.asarray(slots, dtype=np.uint64)
    out = np.zeros(slots.shape + (4,), dtype=np.uint64)
    out[..., 0] = step & MASK
    out[..., 1] = tag
    out[..., 2] = slots
    out[..., 3] = lane
    return out


def to_params(x, kind, t_c):
    """Sampling coordinates -> 16-entry parameter rows (see include/lisatd.h)."""
    x = np.atleast_2d(x)
    p = np.zeros((x.shape[0], 16))
    p[:, 0], p[:, 1] = x[:, 0], x[:, 1]
    if kind == "precessing14":
        for a, th, ph, col in ((2, 3, 4, 2), (5, 6, 7, 5)):
            p[:, col] = x[:, a] * np.sin(x[:, th]) * np.cos(x[:, ph])
            p[:, col + 1] = x[:, a] * np.sin(x[:, th]) * np.sin(x[:, ph])
            p[:, col + 2] = x[:, a] * np.cos(x[:, th])
        p[:, 8], p[:, 9], p[:, 10], p[:, 13], p[:, 12], p[:, 14] = x[:, 8], x[:, 9], x[:, 10], x[:, 11], x[:, 12], x[:, 13]
    elif kind == "aligned10":
        p[:, 4], p[:, 7] = x[:, 2], x[:, 3]
        p[:, 8], p[:, 9], p[:, 10], p[:, 13], p[:, 12], p[:, 14] = x[:, 4], x[:, 5], x[:, 6], x[:, 7], x[:, 8], x[:, 9]
    else:
        raise ValueError(kind)
    p[:, 11] = t_c
    return p


class PTSampler:
    """State X [T][W][d]; logl_fn maps coordinates [n][d] to logL [n]."""

    def __init__(self, logl_fn, lo, hi, n_walkers, n_temps, dim, seed, a=2.0, t_max=10.0):
        self.logl_fn = logl_fn
        self.lo, self.hi = np.asarray(lo, float), np.asarray(hi, float)
        self.W, self.T, self.d, self.a = n_walkers, n_temps, dim, a
        self.key = (seed & MASK, (seed >> 32) & MASK)
        self.beta = np.array([t_max ** (-i / (n_temps - 1)) if n_temps > 1 else 1.0 for i in range(n_temps)])
        self.step_count = 0
        self.acc = self.prop = self.sacc = self.sprop = 0
        self.flow = None
        self.fold = None
        self.walk = 0.0
        self.p_flow = 1.0
        self.flow_exclusive = False
        self.flow2 = None
        self.facc = self.fprop = 0
        self.flow_steps = 0

    def set_flow(self, P, mu, sigma):
        """Attach a flow (oracle.flow parameters; None detaches)."""
        self.flow = None if P is None else (P, np.asarray(mu, float), np.asarray(sigma, float))

    def set_flow_fold(self, index, period=math.pi, start=0.0):
        """Fold coordinate `index` into [start, start + period) for the flow move (index < 0: none)."""
        self.fold = None if index < 0 else (int(index), float(period), float(start))

    def set_flow_mix(self, p_flow):
        """Probability that a step runs the flow move (0: the plain sampler)."""
        self.p_flow = float(p_flow)

    def set_flow_mixture(self, P2, mu2, sigma2, w1):
        """Second flow of a two-component proposal q = w1 q1 + (1 - w1) q2 (None: one flow)."""
        if P2 is None:
            self.flow2 = None
            return
        if not 0.0 < w1 < 1.0:
            raise ValueError("w1 must lie in (0, 1)")
        self.flow2 = (P2, np.asarray(mu2, float), np.asarray(sigma2, float), float(w1))

    def _mix_logq(self, x):
        """log(w1 q1(x) + w2 q2(x)) of folded points x."""
        P, mu, sigma = self.flow
        P2, mu2, sigma2, w1 = self.flow2
        _, l1 = _flow.forward(P, x, mu, sigma)
        _, l2 = _flow.forward(P2, x, mu2, sigma2)
        return np.logaddexp(math.log(w1) + l1, math.log(1.0 - w1) + l2)

    def set_flow_exclusive(self, on):
        """On steps that run the flow move, skip the cold rung's stretch moves."""
        self.flow_exclusive = bool(on)

    def flow_gate(self, s):
        """Whether step s runs the flow move: u < p_flow, u from counter (s, 0x800, 0, 0)."""
        r = philox4x32_10(_ctr(s, TAG_FLOWG, np.array([0])), self.key)
        return bool(u01(r[0, 0]) < self.p_flow)

    def set_flow_walk(self, step):
        """Latent random walk of this step as the flow move (0: independence proposals)."""
        self.walk = float(step)

    def _copies(self, v, i, P):
        """Copies v + k P inside [lo_i, hi_i]: (k_min, count)."""
        a = np.ceil((self.lo[i] - v) / P)
        b = np.floor((self.hi[i] - v) / P)
        return a, np.where(b >= a, b - a + 1, 0).astype(np.int64)

    def flow_normals(self, s, tag=TAG_FLOWZ):
        """Standard normals [W][d] of step s (base samples; the walk's steps with TAG_FLOWW)."""
        W, d = self.W, self.d
        z = np.zeros((W, d))
        k = np.arange(W)
        for q in range((d + 3) // 4):
            r = philox4x32_10(_ctr(s, tag, k, q), self.key)
            for p in (0, 1):
                rad = np.sqrt(-2.0 * np.log(u01(r[:, 2 * p])))
                ph = 2.0 * math.pi * u01(r[:, 2 * p + 1])
                i0 = 4 * q + 2 * p
                if i0 < d:
                    z[:, i0] = rad * np.cos(ph)
                if i0 + 1 < d:
                    z[:, i0 + 1] = rad * np.sin(ph)
        return z

    @staticmethod
    def _log_normal(z):
        acc = np.zeros(z.shape[0])
        for i in range(z.shape[1]):
            acc = acc + z[:, i] * z[:, i]
        return -0.5 * acc - 0.5 * z.shape[1] * math.log(2.0 * math.pi)

    def flow_move(self, s):
        P, mu, sigma = self.flow
        W = self.W
        xf = self.X[0].copy()
        lkx = np.zeros(W)
        out = np.zeros(W, dtype=bool)
        if self.fold is not None:
            i, Pf, c0 = self.fold
            x = self.X[0, :, i]
            xf[:, i] = c0 + ((x - c0) - Pf * np.floor((x - c0) / Pf))
            _, nx = self._copies(xf[:, i], i, Pf)
            lkx = np.where(nx > 0, np.log(np.maximum(nx, 1).astype(np.float64)), 0.0)
        if self.flow2 is not None:
            if self.walk > 0.0:
                raise ValueError("the latent walk takes one flow")
            P2, mu2, sigma2, w1 = self.flow2
            z = self.flow_normals(s)
            y1, _ = _flow.inverse(P, z, mu, sigma)
            y2, _ = _flow.inverse(P2, z, mu2, sigma2)
            rc = philox4x32_10(_ctr(s, TAG_FLOWM, np.arange(W)), self.key)
            y = np.where((u01(rc[:, 0]) < w1)[:, None], y1, y2)
            lqy = self._mix_logq(y)
            lqx = self._mix_logq(xf)
        elif self.walk > 0.0:
            z, lqx = _flow.forward(P, xf, mu, sigma)
            zn = z + self.walk * self.flow_normals(s, TAG_FLOWW)
            lqx = lqx - self._log_normal(z)
            y, lqy = _flow.inverse(P, zn, mu, sigma)
            lqy = lqy - self._log_normal(zn)
        else:
            y, lqy = _flow.inverse(P, self.flow_normals(s), mu, sigma)
            _, lqx = _flow.forward(P, xf, mu, sigma)
        if self.fold is not None:
            i, Pf, c0 = self.fold
            v = y[:, i].copy()
            inwin = (v >= c0) & (v < c0 + Pf)
            km, ny = self._copies(v, i, Pf)
            ny = np.where(inwin, ny, 0)
            ru_c = philox4x32_10(_ctr(s, TAG_FLOWC, np.arange(W)), self.key)
            j = np.minimum(np.floor(u01(ru_c[:, 0]) * ny.astype(np.float64)).astype(np.int64), ny - 1)
            okc = ny > 0
            y[okc, i] = v[okc] + (km[okc] + j[okc].astype(np.float64)) * Pf
            lqy = np.where(okc, lqy - np.log(np.maximum(ny, 1).astype(np.float64)), lqy)
            out = ~okc
        lpy = np.where(out, -np.inf, self.log_prior(y))
        lly = np.asarray(self.logl_fn(y), dtype=np.float64)
        ru = philox4x32_10(_ctr(s, TAG_FLOWU, np.arange(W)), self.key)
        with np.errstate(invalid="ignore"):
            la = self.beta[0] * (lly - self.logl[0]) + (lpy - self.logp[0]) + ((lqx - lkx) - lqy)
            ok = (lpy > -np.inf) & ~np.isnan(lly) & (lly > -np.inf) & ~np.isnan(la) & (np.log(u01(ru[:, 0])) < la)
        self.X[0, ok] = y[ok]
        self.logl[0, ok] = lly[ok]
        self.logp[0, ok] = lpy[ok]
        self.facc += int(ok.sum())
        self.fprop += W
        return ok

    def log_prior(self, x):
        inside = np.all((x >= self.lo) & (x <= self.hi), axis=-1)
        return np.where(inside, 0.0, -np.inf)

    def set_state(self, X):
        self.X = np.array(X, dtype=np.float64).reshape(self.T, self.W, self.d)
        flat = self.X.reshape(-1, self.d)
        self.logp = self.log_prior(flat).reshape(self.T, self.W)
        self.logl = np.asarray(self.logl_fn(flat), dtype=np.float64).reshape(self.T, self.W)
        self.step_count = 0
        self.acc = self.prop = self.sacc = self.sprop = 0
        self.facc = self.fprop = 0
        self.flow_steps = 0

    def step(self):
        T, W, d, half = self.T, self.W, self.d, self.W // 2
        s = self.step_count
        gate = self.flow is not None and self.p_flow > 0.0 and self.flow_gate(s)
        t_first = 1 if gate and self.flow_exclusive else 0
        for h in (0, 1):
            t = np.repeat(np.arange(t_first, T), half)
            k = h * half + np.tile(np.arange(half), T - t_first)
            if t.size == 0:
                continue
            r = philox4x32_10(_ctr(s, TAG_MOVE + h, t * W + k), self.key)
            jj = np.minimum((u01(r[:, 0]) * half).astype(np.int64), half - 1)
            j = (1 - h) * half + jj
            z = ((self.a - 1.0) * u01(r[:, 1]) + 1.0) ** 2 / self.a
            xk, xj = self.X[t, k], self.X[t, j]
            Y = xj + z[:, None] * (xk - xj)
            lpy = self.log_prior(Y)
            lly = np.asarray(self.logl_fn(Y), dtype=np.float64)
            la = (d - 1) * np.log(z) + self.beta[t] * (lly - self.logl[t, k]) + (lpy - self.logp[t, k])
            with np.errstate(invalid="ignore"):
                ok = (lpy > -np.inf) & ~np.isnan(lly) & (lly > -np.inf) & (np.log(u01(r[:, 2])) < la)
            self.X[t[ok], k[ok]] = Y[ok]
            self.logl[t[ok], k[ok]] = lly[ok]
            self.logp[t[ok], k[ok]] = lpy[ok]
            self.acc += int(ok.sum())
            self.prop += ok.size
        if gate:
            self.flow_move(s)
            self.flow_steps += 1
        for i in range(T - 2, -1, -1):
            rr = philox4x32_10(_ctr(s, TAG_SHIFT + i, np.array([0])), self.key)
            shift = int(rr[0, 0] % np.uint64(W))
            k = np.arange(W)
            k2 = (k + shift) % W
            ru = philox4x32_10(_ctr(s, TAG_SWAP + i, k), self.key)
            with np.errstate(invalid="ignore"):
                la = (self.beta[i] - self.beta[i + 1]) * (self.logl[i + 1, k2] - self.logl[i, k])
                ok = np.log(u01(ru[:, 0])) < la
            a_idx, b_idx = k[ok], k2[ok]
            for arr in (self.X, self.logl, self.logp):
                tmp = arr[i, a_idx].copy()
                arr[i, a_idx] = arr[i + 1, b_idx]
                arr[i + 1, b_idx] = tmp
            self.sacc += int(ok.sum())
            self.sprop += W
        self.step_count += 1


def gaussian_logl(mean, icov):
    """Equal-weight mixture of Gaussians sharing one inverse covariance."""
    means = np.atleast_2d(mean)

    def f(x):
        x = np.atleast_2d(x)
        q = np.stack([-0.5 * np.einsum("ni,ij,nj->n", x - m, icov, x - m) for m in means])
        best = q.max(axis=0)
        return best + np.log(np.exp(q - best).sum(axis=0) / len(means))
    return f


def integrated_time(chain, c=5.0):
    """Integrated autocorrelation time per coordinate of chain [steps][walkers][d]
    (autocorrelation averaged over walkers, Sokal's window: smallest M with
    M >= c tau(M))."""
    chain = np.asarray(chain, dtype=np.float64)
    n = chain.shape[0]
    taus = []
    for q in range(chain.shape[2]):
        acf = np.zeros(n)
        for w in range(chain.shape[1]):
            x = chain[:, w, q] - chain[:, w, q].mean()
            f = np.fft.rfft(x, 2 * n)
            r = np.fft.irfft(f * np.conj(f))[:n]
            if r[0] > 0:
                acf += r / r[0]
        acf /= chain.shape[1]
        tau = 2.0 * np.cumsum(acf) - 1.0
        m = np.arange(n)
        ok = m >= c * tau
        M = int(np.argmax(ok)) if np.any(ok) else n - 1
        taus.append(tau[M])
    return np.array(taus)
