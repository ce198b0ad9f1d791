"""PhenomT-form co-precessing modes, FP64 (paper Sec. II.A).  Test infrastructure only.

The paper evaluates the IMRPhenomT family mode by mode as closed-form
functions of time, each time sample independent of the others (Sec. II.A,
first paragraph).  The calibrated IMRPhenomT ansatz and coefficients are not
printed in the paper, so this oracle defines a "PhenomT-form" model with the
same structure, built from public post-Newtonian physics:

* inspiral: TaylorT3 closed form in theta = [eta (t_c - t) / (5 M)]^(-1/8),
  orbital phase Phi(theta) = -theta^-5/eta (1 + a2 theta^2 + a3 theta^3 +
  a4 theta^4) (2PN, with the 1.5PN spin-orbit term), and the orbital
  frequency defined as its exact time derivative;
* merger-ringdown: for t >= t_m the (2,2) frequency is a tanh step
  omega_lo + Delta (1 + tanh(t/w))/2 centred on the peak time t = 0, joined
  C^1 to the inspiral and tending to the (2,2) quasi-normal-mode frequency;
  its phase is the closed-form integral;
* amplitude: leading-order |h22| = 8 sqrt(pi/5) eta (M/D) x, a quadratic cap
  on [t_m, 0] joined C^1 with its maximum at t = 0, and a sech ringdown with
  the quasi-normal-mode damping time for t >= 0;
* higher modes: leading-PN amplitude ratios H_lm(x) times the (2,2)
  envelope, phases m/2 times the (2,2) phase;
* hard start where the (2,2) frequency equals f_low; orbital phase zero at
  f_ref (the reference phase enters only through the line-of-sight rotation).

Agreement with the real IMRPhenomT family is parity unpinned.
"""
import math
import numpy as np

from .phys import C_SI, MTSUN_SI, MPC_SI

# parameter vector layout (one row per template)
P_M1, P_M2 = 0, 1
P_CHI1, P_CHI2 = slice(2, 5), slice(5, 8)
P_DL, P_IOTA, P_PHI, P_TC, P_LAM, P_BETA, P_PSI = 8, 9, 10, 11, 12, 13, 14
N_PARAMS = 16

THETA_MATCH = 0.7          # inspiral / merger matching point in theta
MODES_ALL = ((2, 2), (2, 1), (3, 3), (3, 2), (4, 4))


def real_array(x):
    """x as a float64 array, or as np.longdouble when it already is one.  Every function of
    the time and phase path keeps the caller's precision, so the same code evaluates the
    model in FP64 (the parity target) and in x87 extended precision (the reference that
    measures FP64's own rounding floor)."""
    x = np.asarray(x)
    return x if x.dtype == np.longdouble else np.asarray(x, dtype=np.float64)


def complex_of(x):
    """The complex dtype matching x's real precision."""
    return np.result_type(np.asarray(x).dtype, np.complex64)


def _remnant(eta, m1f, m2f, chi1l, chi2l):
    """Builder-defined remnant spin and mass fraction (parity unpinned)."""
    af = 2.0 * math.sqrt(3.0) * eta - 3.871 * eta ** 2 + 4.028 * eta ** 3 \
        + m1f ** 2 * chi1l + m2f ** 2 * chi2l
    af = min(0.99, max(-0.99, af))
    mf = 1.0 - 0.0484 * (4.0 * eta) ** 2
    return af, mf


def _qnm22(af):
    """(2,2,0) quasi-normal mode: dimensionless frequency and quality factor."""
    w = 1.5251 - 1.1568 * (1.0 - af) ** 0.1292
    q = 0.7 + 1.4187 * (1.0 - af) ** (-0.4990)
    return w, q


class Template:
    """Per-template scalars (hot-path step a1) for the PhenomT-form model."""

    def __init__(self, p, f_low=1e-4, f_ref=1e-4, pn=True, spins_aligned=True, real=np.float64):
        """real: np.float64 (the oracle) or np.longdouble (the extended-precision reference of
        the same model, same FP64 coefficients, for measuring FP64's rounding floor)."""
        R = float if real is np.float64 else real
        tanh = math.tanh if real is np.float64 else np.tanh
        self.real = real
        p = np.asarray(p, dtype=np.float64)
        m1, m2 = R(p[P_M1]), R(p[P_M2])
        self.valid = True
        if not (m1 > 0 and m2 > 0):
            self.valid = False
            m1, m2 = 1.0, 1.0
        M = m1 + m2
        self.M = M
        self.Ms = M * MTSUN_SI
        self.eta = m1 * m2 / M ** 2
        self.delta = (m1 - m2) / M
        self.m1f, self.m2f = m1 / M, m2 / M
        chi1 = np.array(p[P_CHI1], dtype=real)
        chi2 = np.array(p[P_CHI2], dtype=real)
        if np.linalg.norm(chi1) >= 1.0 or np.linalg.norm(chi2) >= 1.0:
            self.valid = False
        self.chi1, self.chi2 = chi1, chi2
        self.chi1l, self.chi2l = R(chi1[2]), R(chi2[2])
        self.DL = R(p[P_DL])
        if not self.DL > 0:
            self.valid = False
            self.DL = 1.0
        self.iota, self.phi_ref = R(p[P_IOTA]), R(p[P_PHI])
        self.tc = R(p[P_TC])
        self.lam, self.beta, self.psi = R(p[P_LAM]), R(p[P_BETA]), R(p[P_PSI])
        self.f_low, self.f_ref = f_low, f_ref
        eta = self.eta
        # TaylorT3 phase coefficients (2PN, spin-orbit at 1.5PN)
        beta_so = sum((113.0 / 12.0 * mf ** 2 + 25.0 / 4.0 * eta) * chi
                      for mf, chi in ((self.m1f, self.chi1l), (self.m2f, self.chi2l)))
        if pn:
            self.a2 = 3715.0 / 8064.0 + 55.0 / 96.0 * eta
            self.a3 = -0.75 * math.pi + 3.0 / 16.0 * beta_so
            self.a4 = 9275495.0 / 14450688.0 + 284875.0 / 258048.0 * eta + 1855.0 / 2048.0 * eta ** 2
        else:
            self.a2 = self.a3 = self.a4 = 0.0
        # matching point: the PN coalescence time sits at the peak, t = 0
        self.theta_m = THETA_MATCH
        self.T = 5.0 * self.Ms / (eta * self.theta_m ** 8)
        self.t_m = -self.T
        self.w22_m = 2.0 * self.omega_orb_theta(self.theta_m)
        self.dw22_m = 2.0 * self.domega_orb_dtheta(self.theta_m) * self.dtheta_dt(self.theta_m)
        # ringdown
        self.af, self.mf = _remnant(eta, self.m1f, self.m2f, self.chi1l, self.chi2l)
        wq, qq = _qnm22(self.af)
        self.w_rd = wq / (self.mf * self.Ms)
        self.tau_rd = 2.0 * qq / self.w_rd
        # tanh step: s (1 - tanh s) = kappa T, larger root
        kappa = self.dw22_m / (self.w_rd - self.w22_m)
        target = kappa * self.T
        if not (self.w_rd > self.w22_m and 0.0 < target < 0.2784):
            self.valid = False
            target = 0.1
        lo, hi = R(0.6392), R(60.0)
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if mid * (1.0 - tanh(mid)) > target:
                lo = mid
            else:
                hi = mid
        s = 0.5 * (lo + hi)
        self.w = self.T / s
        sig_m = 0.5 * (1.0 - tanh(s))
        self.Delta = (self.w_rd - self.w22_m) / (1.0 - sig_m)
        self.w_lo = self.w_rd - self.Delta
        # reference and start points (inspiral only)
        self.theta_ref = self.solve_theta(math.pi * f_ref)
        self.theta_start = self.solve_theta(math.pi * f_low)
        if self.theta_ref is None or self.theta_start is None:
            self.valid = False
            self.theta_ref = self.theta_start = 0.5 * self.theta_m
        self.Phi_ref = self.Phi_theta(self.theta_ref)
        self.t_start = -5.0 * self.Ms / (eta * self.theta_start ** 8)
        self.phi22_m = 2.0 * (self.Phi_theta(self.theta_m) - self.Phi_ref)
        # amplitude
        self.K_amp = 8.0 * math.sqrt(math.pi / 5.0) * eta * self.Ms * C_SI / (self.DL * MPC_SI)
        x_m = (self.Ms * self.w22_m / 2.0) ** (2.0 / 3.0)
        self.A_m = self.K_amp * x_m
        self.dA_m = self.K_amp * (2.0 / 3.0) * x_m * self.dw22_m / self.w22_m
        self.A_p = self.A_m + 0.5 * self.dA_m * self.T

    # --- inspiral pieces -------------------------------------------------
    def Phi_theta(self, th):
        return -(1.0 / self.eta) * th ** -5 * (1.0 + self.a2 * th ** 2 + self.a3 * th ** 3 + self.a4 * th ** 4)

    def omega_orb_theta(self, th):
        # exact d Phi / dt = (d Phi / d theta)(d theta / dt)
        return th ** 3 / (8.0 * self.Ms) * (1.0 + 0.6 * self.a2 * th ** 2 + 0.4 * self.a3 * th ** 3
                                            + 0.2 * self.a4 * th ** 4)

    def domega_orb_dtheta(self, th):
        return (3.0 * th ** 2 + 3.0 * self.a2 * th ** 4 + 2.4 * self.a3 * th ** 5
                + 1.4 * self.a4 * th ** 6) / (8.0 * self.Ms)

    def dtheta_dt(self, th):
        return self.eta * th ** 9 / (40.0 * self.Ms)

    def theta_of_t(self, t):
        """theta(t) = [eta (0 - t) / (5 M)]^(-1/8), model time (peak at t = 0)."""
        return (self.eta * (-real_array(t)) / (5.0 * self.Ms)) ** (-0.125)

    def solve_theta(self, w_orb):
        """Inspiral theta at which the orbital frequency equals w_orb (Newton)."""
        if not w_orb < self.omega_orb_theta(self.theta_m):
            return None
        th = min((8.0 * self.Ms * w_orb) ** (1.0 / 3.0), 0.9 * self.theta_m)
        for _ in range(100):
            d = (self.omega_orb_theta(th) - w_orb) / self.domega_orb_dtheta(th)
            th -= d
            if abs(d) < 1e-16 * th:
                break
        return th

    # --- full (2,2) frequency, phase, amplitude ----------------------------
    def omega22(self, t):
        t = real_array(t)
        out = np.empty_like(t)
        ins = t < self.t_m
        out[ins] = 2.0 * self.omega_orb_theta(self.theta_of_t(t[ins]))
        tm = t[~ins]
        out[~ins] = self.w_lo + 0.5 * self.Delta * (1.0 + np.tanh(tm / self.w))
        return out

    def phi22(self, t):
        t = real_array(t)
        out = np.empty_like(t)
        ins = t < self.t_m
        out[ins] = 2.0 * (self.Phi_theta(self.theta_of_t(t[ins])) - self.Phi_ref)
        tm = t[~ins]
        out[~ins] = (self.phi22_m + (self.w_lo + 0.5 * self.Delta) * (tm - self.t_m)
                     + 0.5 * self.Delta * self.w * (_lncosh(tm / self.w) - _lncosh(self.t_m / self.w)))
        return out

    def x_of_t(self, t):
        """PN parameter x = (M omega22 / 2)^(2/3), continued through merger."""
        return (self.Ms * self.omega22(t) / 2.0) ** (2.0 / 3.0)

    def amp22(self, t):
        t = real_array(t)
        out = np.empty_like(t)
        ins = t < self.t_m
        out[ins] = self.K_amp * self.x_of_t(t[ins])
        mer = (~ins) & (t < 0.0)
        out[mer] = self.A_p - (self.A_p - self.A_m) * (t[mer] / self.t_m) ** 2
        rd = t >= 0.0
        out[rd] = self.A_p / np.cosh(t[rd] / self.tau_rd)
        return out

    def mode_ratio(self, l, m, x):
        """Leading-PN amplitude ratio H_lm(x) / H_22 (complex)."""
        eta, d = self.eta, self.delta
        if (l, m) == (2, 2):
            return np.ones_like(x, dtype=complex_of(x))
        if (l, m) == (2, 1):
            return (1j / 3.0) * d * np.sqrt(x)
        if (l, m) == (3, 3):
            return -0.75j * math.sqrt(15.0 / 14.0) * d * np.sqrt(x)
        if (l, m) == (3, 2):
            return (1.0 / 3.0) * math.sqrt(5.0 / 7.0) * (1.0 - 3.0 * eta) * x + 0j
        if (l, m) == (4, 4):
            return -(8.0 / 9.0) * math.sqrt(5.0 / 7.0) * (1.0 - 3.0 * eta) * x + 0j
        raise ValueError("unsupported mode (%d,%d)" % (l, m))


def _lncosh(z):
    a = np.abs(z)
    return a + np.log1p(np.exp(-2.0 * a)) - math.log(2.0)


def cp_modes(tpl, t_ssb, modes=MODES_ALL):
    """Co-precessing modes h_lm(t) for m > 0 at SSB times t (hot-path step a2).

    h_lm = A22(t) H_lm(x(t)) exp(-i m phi_orb(t)) for t >= t_start, else 0,
    with phi_orb = phi22 / 2.  Negative m follow from h_{l,-m} = (-1)^l conj(h_lm).
    Returns complex array [len(modes)][len(t)].
    """
    t = real_array(t_ssb) - tpl.tc
    out = np.zeros((len(modes), t.size), dtype=complex_of(t))
    on = t >= tpl.t_start
    ts = t[on]
    A = tpl.amp22(ts)
    phi_orb = 0.5 * tpl.phi22(ts)
    x = tpl.x_of_t(ts)
    for i, (l, m) in enumerate(modes):
        out[i, on] = A * tpl.mode_ratio(l, m, x) * np.exp(-1j * m * phi_orb)
    return out
