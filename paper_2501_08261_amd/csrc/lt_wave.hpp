// PhenomT-form waveform on the device: per-template setup (hot-path step a1)
// and per-sample evaluation of the co-precessing modes (a2), the Euler-angle
// quaternion (a3) and the single-sum twist-up to h+, hx (a4).
//
// Model (paper Sec. II.A; the calibrated IMRPhenomT ansatz is not printed, so
// this is a PhenomT-form model built from public post-Newtonian physics):
//  * inspiral: TaylorT3 closed form in theta = [eta (t_c - t)/(5M)]^(-1/8),
//    orbital phase Phi = -theta^-5/eta (1 + a2 theta^2 + a3 theta^3 + a4 theta^4)
//    and its exact time derivative as the orbital frequency;
//  * merger-ringdown (t >= t_m): omega22 = w_lo + Delta (1 + tanh(t/w))/2,
//    C^1-joined at t_m and tending to the (2,2) QNM frequency, phase by its
//    closed-form integral;
//  * amplitude: 8 sqrt(pi/5) eta (M/D) x in the inspiral, a quadratic cap with
//    its maximum at t = 0 on [t_m, 0], a sech ringdown with the QNM damping;
//  * higher modes: leading-PN amplitude ratios, phases m times the orbital phase.
// Precession: single-spin simple precession of L about J, closed forms in
// u = (M omega22 / 2)^(1/3) for alpha, beta, gamma (NNLO-form), constant
// J -> L0 rotation chosen so that the composite rotation is the identity at
// f_ref.  Twist-up: Eq. (2.4) with the rotor Q = conj(q_CP->J) conj(q_J->L0)
// q(phi, iota, 0), quaternions of Eq. (2.5) (normalised), and the
// division-free form of Eq. (2.6): W^l_m = D^l_{m,2} as a polynomial in Q_a, Q_b.
#pragma once
#include "lt_common.hpp"

namespace lt {

// ---------------------------------------------------------------- Wigner W
__host__ __device__ constexpr double fact(int n) { return n <= 1 ? 1.0 : n * fact(n - 1); }
__host__ __device__ constexpr double binom(int n, int k) {
  return (k < 0 || k > n) ? 0.0 : fact(n) / (fact(k) * fact(n - k));
}

// W^L_M(Q) with pa[k] = Qa^k (k <= 8), pb[k] = Qb^k (k <= 6).
template <int L, int M>
__device__ inline cplx wig(const cplx* pa, const cplx* pb) {
  constexpr int rlo = (M - 2) > 0 ? (M - 2) : 0;
  constexpr int rhi = (L - 2) < (L + M) ? (L - 2) : (L + M);
  double pref = __builtin_sqrt(fact(L + 2) * fact(L - 2) / (fact(L + M) * fact(L - M)));
  cplx acc{0.0, 0.0};
#pragma unroll
  for (int rho = rlo; rho <= rhi; ++rho) {
    double coef = ((rho & 1) ? -1.0 : 1.0) * binom(L + M, rho) * binom(L - M, L - 2 - rho);
    cplx t = cmul(cmul(pa[L + M - rho], cconj(pa[L - 2 - rho])), cmul(pb[2 - M + rho], cconj(pb[rho])));
    acc = cadd(acc, cscale(t, coef));
  }
  return cscale(acc, pref);
}

__device__ inline cplx qmul_scalar_first(const double* a, const double* b, double* out) {
  out[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
  out[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
  out[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
  out[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
  return {0.0, 0.0};
}

template <typename A> __device__ inline A sb_neg(A shb, A sd) { return -shb * sd; }

__device__ inline void quat_euler(double alpha, double cos_hb, double sin_hb, double gamma, double* q) {
  double ss, cs, sd, cd;
  sincos(0.5 * (alpha + gamma), &ss, &cs);
  sincos(0.5 * (alpha - gamma), &sd, &cd);
  q[0] = cos_hb * cs;
  q[1] = -sin_hb * sd;
  q[2] = sin_hb * cd;
  q[3] = cos_hb * ss;
}

// sqrt((2l+1)/4pi) for l = 2, 3, 4
constexpr double kY2 = 0.63078313050504001;   // sqrt(5/(4 pi))
constexpr double kY3 = 0.74635266518023080;   // sqrt(7/(4 pi))
constexpr double kY4 = 0.84628437532163447;   // sqrt(9/(4 pi))

// -------------------------------------------------------------- setup (a1)
__device__ inline double lncosh(double z) {
  double a = fabs(z);
  return a + log1p(exp(-2.0 * a)) - 0.69314718055994531;
}

struct Pn {
  double Ms, a2, a3, a4, eta;
  __device__ double w_orb(double th) const {
    double t2 = th * th;
    return th * t2 / (8.0 * Ms) * (1.0 + 0.6 * a2 * t2 + 0.4 * a3 * t2 * th + 0.2 * a4 * t2 * t2);
  }
  __device__ double dw_orb(double th) const {
    double t2 = th * th;
    return (3.0 * t2 + 3.0 * a2 * t2 * t2 + 2.4 * a3 * t2 * t2 * th + 1.4 * a4 * t2 * t2 * t2) / (8.0 * Ms);
  }
  __device__ double Phi(double th) const {
    double t2 = th * th;
    double tm5 = 1.0 / (t2 * t2 * th);
    return -(1.0 / eta) * tm5 * (1.0 + a2 * t2 + a3 * t2 * th + a4 * t2 * t2);
  }
  // inspiral theta where the orbital frequency equals w (Newton); <0 if beyond matching
  __device__ double solve(double w, double th_m) const {
    if (!(w < w_orb(th_m))) return -1.0;
    double th = fmin(cbrt(8.0 * Ms * w), 0.9 * th_m);
    for (int i = 0; i < 100; ++i) {
      double d = (w_orb(th) - w) / dw_orb(th);
      th -= d;
      if (fabs(d) < 1e-16 * th) break;
    }
    return th;
  }
};

// Fills c from one parameter row p[16]; returns 1 if physical.
__device__ inline int setup_template(const double* p, double f_low, double f_ref, double t0, double dt,
                                     TplConst& c) {
  int valid = 1;
  double m1 = p[0], m2 = p[1];
  if (!(m1 > 0.0 && m2 > 0.0)) { valid = 0; m1 = m2 = 1.0; }
  double M = m1 + m2;
  double Ms = M * kMTsun;
  double eta = m1 * m2 / (M * M);
  double m1f = m1 / M, m2f = m2 / M;
  double chi1[3] = {p[2], p[3], p[4]}, chi2[3] = {p[5], p[6], p[7]};
  double n1 = sqrt(chi1[0] * chi1[0] + chi1[1] * chi1[1] + chi1[2] * chi1[2]);
  double n2 = sqrt(chi2[0] * chi2[0] + chi2[1] * chi2[1] + chi2[2] * chi2[2]);
  if (!(n1 < 1.0 && n2 < 1.0)) valid = 0;
  double DL = p[8];
  if (!(DL > 0.0)) { valid = 0; DL = 1.0; }
  double iota = p[9], phi_ref = p[10], lam = p[12], bet = p[13], psi = p[14];
  c.tc = p[11];
  c.Ms = Ms;
  c.eta = eta;
  c.inv_eta = 1.0 / eta;
  c.delta = (m1 - m2) / M;
  c.eta_5M = eta / (5.0 * Ms);
  double chi1l = chi1[2], chi2l = chi2[2];
  double beta_so = (113.0 / 12.0 * m1f * m1f + 25.0 / 4.0 * eta) * chi1l
                 + (113.0 / 12.0 * m2f * m2f + 25.0 / 4.0 * eta) * chi2l;
  Pn pn;
  pn.Ms = Ms;
  pn.eta = eta;
  pn.a2 = 3715.0 / 8064.0 + 55.0 / 96.0 * eta;
  pn.a3 = -0.75 * kPi + 3.0 / 16.0 * beta_so;
  pn.a4 = 9275495.0 / 14450688.0 + 284875.0 / 258048.0 * eta + 1855.0 / 2048.0 * eta * eta;
  c.a2 = pn.a2; c.a3 = pn.a3; c.a4 = pn.a4;
  const double thm = kThetaMatch;
  double thm2 = thm * thm, thm4 = thm2 * thm2;
  double T = 5.0 * Ms / (eta * thm4 * thm4);
  c.t_m = -T;
  double w22m = 2.0 * pn.w_orb(thm);
  double dw22m = 2.0 * pn.dw_orb(thm) * (eta * thm4 * thm4 * thm / (40.0 * Ms));
  // remnant and (2,2,0) QNM
  double af = 2.0 * sqrt(3.0) * eta - 3.871 * eta * eta + 4.028 * eta * eta * eta
            + m1f * m1f * chi1l + m2f * m2f * chi2l;
  af = fmin(0.99, fmax(-0.99, af));
  double mf = 1.0 - 0.0484 * (4.0 * eta) * (4.0 * eta);
  double wq = 1.5251 - 1.1568 * pow(1.0 - af, 0.1292);
  double qq = 0.7 + 1.4187 * pow(1.0 - af, -0.4990);
  double w_rd = wq / (mf * Ms);
  c.tau_rd = 2.0 * qq / w_rd;
  // tanh step: s (1 - tanh s) = kappa T, larger root.  g(s) = s (1 - tanh s) peaks at 0.2784
  // for s = 0.6392 and falls beyond, so the root lies in [0.6392, 60].  Newton steps on
  // f(s) = g(s) - target with 1 - tanh s = 2 e / (1 + e), e = exp(-2 s) (no cancellation at
  // large s) and f'(s) = (1 - tanh s)(1 - s (1 + tanh s)), kept inside a bracket [lo, hi] with
  // f(lo) > 0 > f(hi): a step that leaves it bisects instead.  It starts from the large-s
  // asymptote s = ln(2 s / target) / 2 and stops when the step or the bracket is below 1e-15 s
  // (at most 13 steps over the whole target range; a 64-step bisection took 64 tanh calls).
  double target = dw22m / (w_rd - w22m) * T;
  if (!(w_rd > w22m && target > 0.0 && target < 0.2784)) { valid = 0; target = 0.1; }
  double s;
  {
    double lo = 0.6392, hi = 60.0;
    s = 0.5 * log(2.0 / target);
    s = fmin(fmax(0.5 * log(2.0 * s / target), 0.7), 59.0);
    for (int i = 0; i < 100; ++i) {
      const double e = exp(-2.0 * s);
      const double omt = 2.0 * e / (1.0 + e);
      const double f = s * omt - target;
      if (f > 0.0) lo = s; else hi = s;
      double sn = s - f / (omt * (1.0 - s * (2.0 - omt)));
      if (fabs(sn - s) <= 1e-15 * s) { s = sn; break; }
      if (hi - lo <= 1e-15 * hi) { s = 0.5 * (lo + hi); break; }
      if (!(sn > lo && sn < hi)) sn = 0.5 * (lo + hi);
      s = sn;
    }
  }
  c.wt = T / s;
  c.inv_wt = 1.0 / c.wt;
  double sig_m = 0.5 * (1.0 - tanh(s));
  c.Delta = (w_rd - w22m) / (1.0 - sig_m);
  c.w_lo = w_rd - c.Delta;
  c.lncosh_tm = lncosh(c.t_m * c.inv_wt);
  double th_ref = pn.solve(kPi * f_ref, thm);
  double th_st = pn.solve(kPi * f_low, thm);
  if (th_ref < 0.0 || th_st < 0.0) { valid = 0; th_ref = th_st = 0.5 * thm; }
  c.Phi_ref = pn.Phi(th_ref);
  double ts2 = th_st * th_st, ts4 = ts2 * ts2;
  c.t_start = -5.0 * Ms / (eta * ts4 * ts4);
  c.phi22_m = 2.0 * (pn.Phi(thm) - c.Phi_ref);
  // amplitude
  c.K_amp = 8.0 * sqrt(kPi / 5.0) * eta * Ms * kC / (DL * kMpc);
  double xm = pow(Ms * w22m / 2.0, 2.0 / 3.0);
  c.A_m = c.K_amp * xm;
  double dAm = c.K_amp * (2.0 / 3.0) * xm * dw22m / w22m;
  c.A_p = c.A_m + 0.5 * dAm * T;
  double d = c.delta;
  c.r21 = d / 3.0;                                  // times i
  c.r33 = -0.75 * sqrt(15.0 / 14.0) * d;            // times i
  c.r32 = (1.0 / 3.0) * sqrt(5.0 / 7.0) * (1.0 - 3.0 * eta);
  c.r44 = -(8.0 / 9.0) * sqrt(5.0 / 7.0) * (1.0 - 3.0 * eta);
  // precession constants
  double S[3];
  for (int i = 0; i < 3; ++i) S[i] = chi1[i] * m1f * m1f + chi2[i] * m2f * m2f;
  double Sp = sqrt(S[0] * S[0] + S[1] * S[1]);
  c.sig = S[2] / eta;
  c.vsig2 = (Sp / eta) * (Sp / eta);
  double qs = fmin(m1f, m2f) / fmax(m1f, m2f);
  c.Cp = 5.0 * (4.0 + 3.0 * qs) / 256.0;
  double u_ref = cbrt(kPi * Ms * f_ref);
  double J[3] = {S[0], S[1], eta / u_ref + S[2]};
  double beta_ref = atan2(sqrt(J[0] * J[0] + J[1] * J[1]), J[2]);
  double phi_J = atan2(J[1], J[0]);
  c.kappa = phi_J - kPi;
  double ur2 = u_ref * u_ref, ur3 = ur2 * u_ref;
  c.a_ref = -c.Cp * ((2.0 / 3.0) / ur3 + c.sig / ur2);
  c.g_ref = 2.0 * c.Cp * (1.0 / (3.0 * ur3) + 0.5 * c.sig / ur2 - 0.5 * c.vsig2 / u_ref);
  // constant rotor Qc = conj(q_J->L0) q(phi_ref, iota, 0), q_J->L0 = q(kappa, -beta_ref, 0)
  double q0[4], ql[4];
  quat_euler(c.kappa, cos(-0.5 * beta_ref), sin(-0.5 * beta_ref), 0.0, q0);
  quat_euler(phi_ref, cos(0.5 * iota), sin(0.5 * iota), 0.0, ql);
  double q0c[4] = {q0[0], -q0[1], -q0[2], -q0[3]};
  qmul_scalar_first(q0c, ql, c.Qc);
  // polarisation rotation and the aligned-spin harmonics times exp(2 i psi)
  double s2p, c2p;
  sincos(2.0 * psi, &s2p, &c2p);
  c.e2ipsi[0] = c2p;
  c.e2ipsi[1] = s2p;
  {
    cplx Qa{ql[0], ql[3]}, Qb{ql[2], ql[1]};
    cplx pa[9], pb[7];
    pa[0] = {1.0, 0.0};
    pb[0] = {1.0, 0.0};
    for (int k = 1; k < 9; ++k) pa[k] = cmul(pa[k - 1], Qa);
    for (int k = 1; k < 7; ++k) pb[k] = cmul(pb[k - 1], Qb);
    cplx e{c2p, s2p};
    cplx Yp[5] = {cscale(wig<2, 2>(pa, pb), kY2), cscale(wig<2, 1>(pa, pb), kY2), cscale(wig<3, 3>(pa, pb), kY3),
                  cscale(wig<3, 2>(pa, pb), kY3), cscale(wig<4, 4>(pa, pb), kY4)};
    cplx Ym[5] = {cscale(wig<2, -2>(pa, pb), kY2), cscale(wig<2, -1>(pa, pb), kY2),
                  cscale(wig<3, -3>(pa, pb), -kY3), cscale(wig<3, -2>(pa, pb), -kY3),
                  cscale(wig<4, -4>(pa, pb), kY4)};
    for (int i = 0; i < 5; ++i) {
      cplx a = cmul(Yp[i], e), b = cmul(Ym[i], e);
      c.cp[i][0] = a.re; c.cp[i][1] = a.im;
      c.cm[i][0] = b.re; c.cm[i][1] = b.im;
    }
  }
  // sky basis, Eq. (2.7)
  double cl = cos(lam), sl = sin(lam), cb = cos(bet), sb = sin(bet);
  c.k[0] = -cb * cl; c.k[1] = -cb * sl; c.k[2] = -sb;
  c.v[0] = -sb * cl; c.v[1] = -sb * sl; c.v[2] = cb;
  c.u[0] = sl; c.u[1] = -cl; c.u[2] = 0.0;
  c.valid = valid ? 1.0 : 0.0;
  c.n_start = ceil((c.tc + c.t_start - t0) / dt);
  return valid;
}

// ------------------------------------------------------ per-sample evaluation
// FP64 part (phase, frequency, time): returns false before the f_low start.
//   phi : orbital phase (FP64, unreduced)
//   msw : M omega_orb;  v = msw^(-1/3) = 1/u,  u = (M omega_orb)^(1/3), x = u^2
//   amp : A22 in the merger-ringdown (inspiral: A22 = K_amp x)
// theta = y^(-1/8) and v are seeded in FP32 and refined by NEWTON steps of
// the multiplication-only iterations th <- th (9 - y th^8)/8 and
// v <- v (4 - msw v^3)/3 (each squares the relative error).
template <int NEWTON>
__device__ inline bool phase_state(const TplConst& c, double t, double& phi, double& msw, double& v, double& amp,
                                   bool& insp) {
  double tau = t - c.tc;
  if (tau < c.t_start) return false;
  if (tau < c.t_m) {
    double y = c.eta_5M * (-tau);
    float yf = (float)y;
    double th = (double)__builtin_amdgcn_sqrtf(__builtin_amdgcn_sqrtf(__builtin_amdgcn_rsqf(yf)));
#pragma unroll
    for (int k = 0; k < NEWTON; ++k) {
      double t2 = th * th, t4 = t2 * t2;
      th = th * (9.0 - y * (t4 * t4)) * 0.125;
    }
    double t2 = th * th, t3 = t2 * th;
    phi = -c.inv_eta * y * t3 * (1.0 + c.a2 * t2 + c.a3 * t3 + c.a4 * t2 * t2) - c.Phi_ref;
    msw = 0.125 * t3 * (1.0 + 0.6 * c.a2 * t2 + 0.4 * c.a3 * t3 + 0.2 * c.a4 * t2 * t2);
    insp = true;
    amp = 0.0;
  } else {
    double z = tau * c.inv_wt;
    double w22 = c.w_lo + 0.5 * c.Delta * (1.0 + tanh(z));
    double phi22 = c.phi22_m + (c.w_lo + 0.5 * c.Delta) * (tau - c.t_m) + 0.5 * c.Delta * c.wt * (lncosh(z) - c.lncosh_tm);
    phi = 0.5 * phi22;
    msw = c.Ms * 0.5 * w22;
    insp = false;
    if (tau < 0.0) {
      double r = tau / c.t_m;
      amp = c.A_p - (c.A_p - c.A_m) * r * r;
    } else {
      amp = c.A_p / cosh(tau / c.tau_rd);
    }
  }
  double vv = (double)__builtin_amdgcn_exp2f(-0.33333333f * __builtin_amdgcn_logf((float)msw));
#pragma unroll
  for (int k = 0; k < NEWTON; ++k) vv = vv * (4.0 - msw * (vv * vv * vv)) * (1.0 / 3.0);
  v = vv;
  return true;
}

template <typename A> struct cx { A re, im; };
template <typename A> __device__ inline cx<A> xmul(cx<A> a, cx<A> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename A> __device__ inline cx<A> xadd(cx<A> a, cx<A> b) { return {a.re + b.re, a.im + b.im}; }
template <typename A> __device__ inline cx<A> xsc(cx<A> a, A s) { return {a.re * s, a.im * s}; }
template <typename A> __device__ inline cx<A> xconj(cx<A> a) { return {a.re, -a.im}; }
// a * b + conj(a) * c
template <typename A> __device__ inline cx<A> pair_sum(cx<A> a, cx<A> b, cx<A> c) {
  return {a.re * (b.re + c.re) - a.im * (b.im - c.im), a.re * (b.im + c.im) + a.im * (b.re - c.re)};
}

// sin / cos of an FP64 phase in arithmetic type A
__device__ inline void sincos_a(double x, double& s, double& c) { sincos(x, &s, &c); }
// FP32 sin / cos of an FP64 phase: x = q pi/2 + r with q = rint(2x / pi), r taken in FP64
// (two-part pi/2) and rounded to FP32, |r| <= pi/4; sin r and cos r from their Taylor series
// through r^9 and r^10 (the first omitted terms are below 3e-9 there), then the quadrant
// q mod 4 maps them onto sin x and cos x.  Valid for |x| < 2^31 pi/2.
__device__ inline void sincos_a(double x, float& s, float& c) {
  const double q = rint(x * 0.63661977236758134308);
  const float r = (float)fma(-q, 6.1232339957367660360e-17, fma(-q, 1.5707963267948966192, x));
  const int k = (int)q;
  const float r2 = r * r;
  float sp = fmaf(r2, (float)(1.0 / 362880.0), (float)(-1.0 / 5040.0));
  sp = fmaf(r2, sp, (float)(1.0 / 120.0));
  sp = fmaf(r2, sp, (float)(-1.0 / 6.0));
  const float sr = fmaf(r * r2, sp, r);
  float cr = fmaf(r2, (float)(-1.0 / 3628800.0), (float)(1.0 / 40320.0));
  cr = fmaf(r2, cr, (float)(-1.0 / 720.0));
  cr = fmaf(r2, cr, (float)(1.0 / 24.0));
  cr = fmaf(r2, cr, -0.5f);
  cr = fmaf(r2, cr, 1.0f);
  // quadrants 1, 2, 3: (cos r, -sin r), (-sin r, -cos r), (-cos r, sin r)
  float ss = (k & 1) ? cr : sr, cc = (k & 1) ? sr : cr;
  s = (k & 2) ? -ss : ss;
  c = ((k + 1) & 2) ? -cc : cc;
}
__device__ inline double rsqrt_a(double x) { return 1.0 / sqrt(x); }
__device__ inline float rsqrt_a(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ inline double sqrt_a(double x) { return sqrt(x); }
__device__ inline float sqrt_a(float x) { return __builtin_amdgcn_sqrtf(x); }   // 1 ulp

template <typename A> struct NewtonSteps;
template <> struct NewtonSteps<double> { static constexpr int n = 2; };
template <> struct NewtonSteps<float> { static constexpr int n = 1; };

// h+ - i hx at SSB time t including exp(2 i psi); zero before the start.
// Phase, frequency and the Euler-angle phases are FP64; amplitudes, the
// quaternion, the Wigner-D polynomials and the mode sum are in type A.
// The Wigner-D polynomials of Eq. (2.6) (division-free reading) reduce, with
// a = Q_a, b = Q_b, |a|^2 = A2, |b|^2 = B2, to
//   W2,2 = a^4, W2,1 = 2 a^3 b, W2,-1 = 2 a b^3, W2,-2 = b^4,
//   W3,3 = -sqrt6 a^5 conj(b), W3,2 = a^4 (A2 - 5 B2), W3,-2 = b^4 (5 A2 - B2),
//   W3,-3 = sqrt6 conj(a) b^5, W4,4 = 2 sqrt7 a^6 conj(b)^2, W4,-4 = 2 sqrt7 conj(a)^2 b^6.
template <typename A, bool PREC>
__device__ __attribute__((always_inline)) inline cx<A> polarization_t(const TplConst& c, int mode_mask, double t) {
  double phi, msw, vd, ampd;
  bool insp;
  if (!phase_state<NewtonSteps<A>::n>(c, t, phi, msw, vd, ampd, insp)) return {(A)0, (A)0};
  const double ud = msw * vd * vd;          // (M omega_orb)^(1/3)
  const A u = (A)ud;
  const A x = u * u;
  const A amp = insp ? (A)c.K_amp * x : (A)ampd;
  A sphi, cphi;
  sincos_a(phi, sphi, cphi);
  cx<A> h[5];
  {
    cx<A> E1{cphi, -sphi};
    cx<A> E2 = xmul(E1, E1);
    A a21 = amp * (A)c.r21 * u, a33 = amp * (A)c.r33 * u;
    h[0] = xsc(E2, amp);
    h[1] = {-a21 * E1.im, a21 * E1.re};
    cx<A> E3 = xmul(E2, E1);
    h[2] = {-a33 * E3.im, a33 * E3.re};
    h[3] = xsc(E2, amp * (A)c.r32 * x);
    h[4] = xsc(xmul(E2, E2), amp * (A)c.r44 * x);
  }
  cx<A> acc{(A)0, (A)0};
  if (!PREC) {
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      if (mode_mask & (1 << i)) {
        cx<A> a{(A)c.cp[i][0], (A)c.cp[i][1]}, b{(A)c.cm[i][0], (A)c.cm[i][1]};
        acc = xadd(acc, xadd(xmul(h[i], a), xmul(xconj(h[i]), b)));
      }
    }
    return acc;
  }
  // Euler angles (NNLO-form) with v = 1/u
  const double iu2 = vd * vd, iu3 = iu2 * vd;
  const double alpha = -c.Cp * ((2.0 / 3.0) * iu3 + c.sig * iu2) - c.a_ref;
  const double gamma = -c.kappa + 2.0 * c.Cp * ((1.0 / 3.0) * iu3 + 0.5 * c.sig * iu2 - 0.5 * c.vsig2 * vd) - c.g_ref;
  const A a1 = (A)1 + (A)c.sig * u;
  const A cb = a1 * rsqrt_a(a1 * a1 + (A)c.vsig2 * x);
  const A chb = sqrt_a((A)0.5 * ((A)1 + cb));
  const A omc = (A)0.5 * ((A)1 - cb);
  const A shb = sqrt_a(omc > (A)0 ? omc : (A)0);
  A ss, cs, sd, cd;
  sincos_a(0.5 * (alpha + gamma), ss, cs);
  sincos_a(0.5 * (alpha - gamma), sd, cd);
  // q1 = q(alpha, beta, gamma) (Eq. 2.5, normalised); Q = conj(q1) Qc
  const A w1 = chb * cs, x1 = -shb * sd, y1 = shb * cd, z1 = chb * ss;
  const A qw = (A)c.Qc[0], qx = (A)c.Qc[1], qy = (A)c.Qc[2], qz = (A)c.Qc[3];
  const A Q0 = w1 * qw + x1 * qx + y1 * qy + z1 * qz;
  const A Q1 = w1 * qx - x1 * qw - y1 * qz + z1 * qy;
  const A Q2 = w1 * qy + x1 * qz - y1 * qw - z1 * qx;
  const A Q3 = w1 * qz - x1 * qy + y1 * qx - z1 * qw;
  const cx<A> a{Q0, Q3}, b{Q2, Q1};
  const A A2 = Q0 * Q0 + Q3 * Q3, B2 = Q2 * Q2 + Q1 * Q1;
  const cx<A> a2 = xmul(a, a), b2 = xmul(b, b);
  const cx<A> a4 = xmul(a2, a2), b4 = xmul(b2, b2);
  const A y2 = (A)kY2, y3 = (A)kY3, y4 = (A)kY4;
  if (mode_mask & 1)   // (2, +-2)
    acc = xadd(acc, xsc(pair_sum(h[0], a4, b4), y2));
  if (mode_mask & 2) { // (2, +-1)
    cx<A> ab = xmul(a, b);
    acc = xadd(acc, xsc(pair_sum(h[1], xmul(a2, ab), xmul(b2, ab)), (A)2 * y2));
  }
  if (mode_mask & 4) { // (3, +-3): h33 W3,3 + (-1) conj(h33) W3,-3
    const A s6 = (A)2.44948974278317809820 * y3;
    cx<A> p = xmul(xmul(a4, a), xconj(b)), q = xmul(xmul(b4, b), xconj(a));
    acc = xadd(acc, xsc(pair_sum(h[2], p, q), -s6));
  }
  if (mode_mask & 8) { // (3, +-2)
    cx<A> p = xsc(a4, A2 - (A)5 * B2), q = xsc(b4, -((A)5 * A2 - B2));
    acc = xadd(acc, xsc(pair_sum(h[3], p, q), y3));
  }
  if (mode_mask & 16) { // (4, +-4)
    const A s7 = (A)5.29150262212918118100 * y4;
    cx<A> p = xmul(xmul(a4, a2), xconj(b2)), q = xmul(xmul(b4, b2), xconj(a2));
    acc = xadd(acc, xsc(pair_sum(h[4], p, q), s7));
  }
  return xmul(acc, cx<A>{(A)c.e2ipsi[0], (A)c.e2ipsi[1]});
}

// co-precessing modes (m > 0, order 22, 21, 33, 32, 44) in FP64
__device__ inline bool cp_modes_fp64(const TplConst& c, double t, cplx* h) {
  double phi, msw, vd, ampd;
  bool insp;
  if (!phase_state<2>(c, t, phi, msw, vd, ampd, insp)) return false;
  double u = msw * vd * vd, x = u * u;
  double amp = insp ? c.K_amp * x : ampd;
  double sphi, cphi;
  sincos(phi, &sphi, &cphi);
  cplx E1{cphi, -sphi};
  cplx E2 = cmul(E1, E1), E3 = cmul(E2, E1), E4 = cmul(E2, E2);
  double a21 = amp * c.r21 * u, a33 = amp * c.r33 * u;
  h[0] = cscale(E2, amp);
  h[1] = {-a21 * E1.im, a21 * E1.re};
  h[2] = {-a33 * E3.im, a33 * E3.re};
  h[3] = cscale(E2, amp * c.r32 * x);
  h[4] = cscale(E4, amp * c.r44 * x);
  return true;
}

}  // namespace lt
