"""Precession twist-up, FP64 (paper Sec. II.A, Eqs. 2.1-2.6).  Test infrastructure only.

Conventions fixed here (readings of the paper, listed in the design notes):

* Quaternions are Hamilton quaternions (w, x, y, z); R(q1 q2) = R(q1) R(q2)
  and a unit q acts on vectors as v -> q v conj(q).  The Euler-to-quaternion
  map of Eq. (2.5) printed without its 1/sqrt(2) normalisation is read as
  q = q_z(alpha) q_y(beta) q_z(gamma), i.e. the z-y-z rotation
  R_z(alpha) R_y(beta) R_z(gamma) (checked against the matrix product).
* Eq. (2.6) is read with the roles of m and m' swapped and |Q|^2 expanded,
  giving the division-free polynomial W^l_m(Q_a, Q_b) = D^l_{m,2}.
* The Wigner matrices in Eqs. (2.1)-(2.2) are taken in the convention
  D^l_{m m'}(a, b, g) = exp(i m a) d^l_{m m'}(b) exp(i m' g) (so that D* is
  the textbook active-rotation matrix), with the textbook Wigner small-d.
* The -2 spin-weighted harmonics of Eq. (2.3) are the LAL-convention
  -2Y_lm(iota, phi) = sqrt((2l+1)/4pi) d^l_{m,2}(iota) exp(i m phi).
* The polarisation angle rotates h+ - i hx -> exp(2 i psi)(h+ - i hx).
"""
import math
import numpy as np

from .waveform import cp_modes, complex_of, real_array, MODES_ALL


# ---------------------------------------------------------------- quaternions
def quat_mul(a, b):
    """Hamilton product of quaternion arrays [..., 4]."""
    a, b = np.asarray(a), np.asarray(b)
    w1, x1, y1, z1 = a[..., 0], a[..., 1], a[..., 2], a[..., 3]
    w2, x2, y2, z2 = b[..., 0], b[..., 1], b[..., 2], b[..., 3]
    return np.stack([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2], axis=-1)


def quat_conj(q):
    q = np.array(real_array(q))
    q[..., 1:] *= -1.0
    return q


def quat_from_euler(alpha, beta, gamma):
    """Normalised Eq. (2.5): q for the z-y-z rotation R_z(alpha) R_y(beta) R_z(gamma)."""
    alpha, beta, gamma = np.broadcast_arrays(real_array(alpha), real_array(beta), real_array(gamma))
    cb, sb = np.cos(0.5 * beta), np.sin(0.5 * beta)
    sp, dm = 0.5 * (alpha + gamma), 0.5 * (alpha - gamma)
    return np.stack([cb * np.cos(sp), -sb * np.sin(dm), sb * np.cos(dm), cb * np.sin(sp)], axis=-1)


def quat_to_matrix(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def rot_z(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def rot_y(b):
    c, s = math.cos(b), math.sin(b)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


# --------------------------------------------------------------- Wigner-D
def wigner_small_d(l, mp, m, beta):
    """Textbook Wigner small-d d^l_{mp,m}(beta) (Wigner's sum formula)."""
    beta = np.asarray(beta, dtype=np.float64)
    c, s = np.cos(0.5 * beta), np.sin(0.5 * beta)
    f = math.factorial
    pref = math.sqrt(f(l + mp) * f(l - mp) * f(l + m) * f(l - m))
    out = np.zeros_like(beta)
    for k in range(0, 2 * l + 1):
        a1, a2, a3, a4 = l + m - k, k, l - k - mp, k - m + mp
        if min(a1, a2, a3, a4) < 0:
            continue
        out = out + ((-1) ** (k - m + mp) * pref / (f(a1) * f(a2) * f(a3) * f(a4))
                     * c ** (2 * l - 2 * k + m - mp) * s ** (2 * k - m + mp))
    return out


def wigner_D(l, m, mp, alpha, beta, gamma):
    """D^l_{m m'} in the convention of Eqs. (2.1)-(2.2) (see module docstring)."""
    return np.exp(1j * m * np.asarray(alpha)) * wigner_small_d(l, m, mp, beta) \
        * np.exp(1j * mp * np.asarray(gamma))


def sYlm_m2(l, m, iota, phi):
    """-2Y_lm(iota, phi) in the LAL convention, from the Wigner small-d."""
    return math.sqrt((2 * l + 1) / (4 * math.pi)) * wigner_small_d(l, m, 2, iota) \
        * np.exp(1j * m * np.asarray(phi))


def W_lm(l, m, Qa, Qb):
    """Division-free reading of Eq. (2.6): D^l_{m,2} as a polynomial in Q_a, Q_b."""
    f = math.factorial
    pref = math.sqrt(f(l + 2) * f(l - 2) / (f(l + m) * f(l - m)))
    out = 0.0 + 0.0j
    for rho in range(max(0, m - 2), min(l - 2, l + m) + 1):
        coef = (-1) ** rho * math.comb(l + m, rho) * math.comb(l - m, l - 2 - rho)
        out = out + coef * Qa ** (l + m - rho) * np.conj(Qa) ** (l - 2 - rho) \
            * Qb ** (2 - m + rho) * np.conj(Qb) ** rho
    return pref * out


def Q_ab(q):
    """Q_a = q0 + i q3, Q_b = q2 + i q1 (Eq. 2.6)."""
    q = np.asarray(q)
    return q[..., 0] + 1j * q[..., 3], q[..., 2] + 1j * q[..., 1]


# ------------------------------------------------------ precession (NNLO-form)
class Precession:
    """Builder-defined single-spin precession angles (reading of the NNLO
    prescription, which the paper cites but does not print; parity unpinned).

    With S = S1 + S2 (units M^2) split along / across L at f_ref,
    sigma = S_l/eta, varsigma = S_perp/eta and u = (M omega22/2)^(1/3):
      cos beta(u) = (1 + sigma u) / sqrt((1 + sigma u)^2 + varsigma^2 u^2)
      alpha(u)    = a(u) - a(u_ref),  a(u) = -C (2/3 u^-3 + sigma u^-2)
      gamma(u)    = -kappa + g(u) - g(u_ref),
                    g(u) = 2C (u^-3/3 + sigma u^-2/2 - varsigma^2 u^-1/2)
    with C = 5(4 + 3q)/256 (leading-order simple precession of L about J,
    gamma from the minimal-rotation condition truncated at the order shown).
    The constant J -> L0 rotation is R_z(kappa) R_y(-beta_ref) with
    kappa = phi_J - pi, so that the composite rotation at f_ref is the identity.
    """

    def __init__(self, tpl):
        self.tpl = tpl
        fp64 = tpl.real is np.float64
        R = float if fp64 else tpl.real
        hypot, atan2 = (math.hypot, math.atan2) if fp64 else (np.hypot, np.arctan2)
        S = tpl.chi1 * tpl.m1f ** 2 + tpl.chi2 * tpl.m2f ** 2
        eta = tpl.eta
        self.Sl = R(S[2])
        self.Sp = hypot(R(S[0]), R(S[1]))
        self.sig = self.Sl / eta
        self.vsig = self.Sp / eta
        qs = min(tpl.m1f, tpl.m2f) / max(tpl.m1f, tpl.m2f)
        self.C = 5.0 * (4.0 + 3.0 * qs) / 256.0
        self.u_ref = (math.pi * tpl.Ms * tpl.f_ref) ** (1.0 / 3.0)
        J = np.array([S[0], S[1], eta / self.u_ref + S[2]])
        self.beta_ref = atan2(hypot(J[0], J[1]), J[2])
        self.phi_J = atan2(J[1], J[0])
        self.kappa = self.phi_J - math.pi
        self.a_ref = self.a_of_u(self.u_ref)
        self.g_ref = self.g_of_u(self.u_ref)

    def a_of_u(self, u):
        return -self.C * ((2.0 / 3.0) * u ** -3 + self.sig * u ** -2)

    def g_of_u(self, u):
        return 2.0 * self.C * (u ** -3 / 3.0 + 0.5 * self.sig * u ** -2 - 0.5 * self.vsig ** 2 / u)

    def cos_beta(self, u):
        a = 1.0 + self.sig * u
        return a / np.sqrt(a * a + (self.vsig * u) ** 2)

    def angles(self, t_model):
        u = (self.tpl.Ms * self.tpl.omega22(t_model) / 2.0) ** (1.0 / 3.0)
        alpha = self.a_of_u(u) - self.a_ref
        gamma = -self.kappa + self.g_of_u(u) - self.g_ref
        cb = np.clip(self.cos_beta(u), -1.0, 1.0)
        return alpha, np.arccos(cb), gamma, cb

    def q_J_L0(self):
        return quat_from_euler(self.kappa, -self.beta_ref, 0.0)


def _modes_with_negative(tpl, t, modes):
    """List of (l, m, h_lm(t)) including m < 0 via h_{l,-m} = (-1)^l conj(h_lm)."""
    hp = cp_modes(tpl, t, modes)
    out = []
    for i, (l, m) in enumerate(modes):
        out.append((l, m, hp[i]))
        out.append((l, -m, (-1) ** l * np.conj(hp[i])))
    return out


def _apply_psi(tpl, h):
    return np.exp(2j * tpl.psi) * h


def polarizations(tpl, t_ssb, modes=MODES_ALL, precessing=False):
    """h+ and hx at SSB times via the single-sum Eq. (2.4) (hot-path steps a3-a4).

    h+ - i hx = sum_{l, m} h^CP_lm sqrt((2l+1)/4pi) W^l_m(Q(t)), with the
    composite rotor Q = conj(q_CP->J(t)) conj(q_J->L0) q(phi, iota, 0).
    """
    t = real_array(t_ssb)
    q_los = quat_from_euler(tpl.phi_ref, tpl.iota, 0.0)
    if precessing:
        pr = Precession(tpl)
        al, be, ga, _ = pr.angles(t - tpl.tc)
        q1 = quat_from_euler(al, be, ga)
        Q = quat_mul(quat_mul(quat_conj(q1), quat_conj(pr.q_J_L0())), q_los)
    else:
        Q = np.broadcast_to(q_los, t.shape + (4,))
    Qa, Qb = Q_ab(Q)
    h = np.zeros(t.shape, dtype=complex_of(t))
    for l, m, hlm in _modes_with_negative(tpl, t, modes):
        h = h + hlm * math.sqrt((2 * l + 1) / (4 * math.pi)) * W_lm(l, m, Qa, Qb)
    h = _apply_psi(tpl, h)
    return h.real, -h.imag


def polarizations_explicit(tpl, t_ssb, modes=MODES_ALL, precessing=False):
    """h+ and hx via the explicit two-rotation sums, Eqs. (2.1)-(2.3).

    Only used to cross-check the single-sum path (it does the m' sums and the
    two rotations literally with the Wigner matrices of this module).
    """
    t = np.asarray(t_ssb, dtype=np.float64)
    hcp = {}
    for l, m, hlm in _modes_with_negative(tpl, t, modes):
        hcp[(l, m)] = hlm
    ells = sorted({l for l, _ in modes})
    if precessing:
        pr = Precession(tpl)
        al, be, ga, _ = pr.angles(t - tpl.tc)
        a0, b0, g0 = pr.kappa, -pr.beta_ref, 0.0
    h = np.zeros(t.shape, dtype=np.complex128)
    for l in ells:
        cp = {m: hcp.get((l, m), np.zeros(t.shape, complex)) for m in range(-l, l + 1)}
        if precessing:
            hJ = {m: sum(np.conj(wigner_D(l, m, mp, al, be, ga)) * cp[mp] for mp in range(-l, l + 1))
                  for m in range(-l, l + 1)}
            hL0 = {m: sum(np.conj(wigner_D(l, m, mp, a0, b0, g0)) * hJ[mp] for mp in range(-l, l + 1))
                   for m in range(-l, l + 1)}
        else:
            hL0 = cp
        for m in range(-l, l + 1):
            h = h + hL0[m] * sYlm_m2(l, m, tpl.iota, tpl.phi_ref)
    h = _apply_psi(tpl, h)
    return h.real, -h.imag
