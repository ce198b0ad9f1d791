// Shared device-side definitions of liblisatd: per-template constants, complex
// helpers and physical constants.  Included by every .hip translation unit.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lt {

constexpr double kC = 299792458.0;                 // speed of light [m/s]
constexpr double kMTsun = 4.925490947641267e-06;   // G Msun / c^3 [s]
constexpr double kMpc = 3.085677581491367e22;      // [m]
constexpr double kAU = 1.495978707e11;             // [m]
constexpr double kYear = 31558149.763545603;       // sidereal year [s]
constexpr double kPi = 3.14159265358979323846;
constexpr double kThetaMatch = 0.7;                // inspiral / merger matching point

// Per-template constants (hot-path step a1), produced by the setup kernel and
// read by every per-sample kernel.  All FP64.
struct TplConst {
  // masses and PN phasing
  double Ms, eta, inv_eta, delta, a2, a3, a4, eta_5M;   // eta_5M = eta / (5 Ms)
  double Phi_ref, t_start, tc, t_m;
  // merger-ringdown
  double w_lo, Delta, wt, inv_wt, lncosh_tm, phi22_m, tau_rd, pad0;
  // amplitude and mode ratios
  double K_amp, A_m, A_p, r21, r33, r32, r44, pad1;
  // precession (NNLO-form angles) and the constant rotor conj(q_J->L0) q(phi, iota, 0)
  double Cp, sig, vsig2, a_ref, g_ref, kappa, pad2, pad3;
  double Qc[4];
  // aligned-spin projection coefficients: h = sum_m h_lm cp + conj(h_lm) cm
  double cp[5][2], cm[5][2];
  double e2ipsi[2];
  // sky basis of Eq. (2.7)
  double k[3], u[3], v[3];
  double valid;          // 1 valid, 0 unphysical
  double n_start;        // first grid index at or after the f_low start (may be < 0 or > n)
  double pad4[5];
};
// include/lisatd.h states this size (per-template scratch of the likelihood)
static_assert(sizeof(TplConst) == 624, "set-up constants: 78 doubles per template");

struct cplx { double re, im; };
__device__ __host__ inline cplx cmul(cplx a, cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __host__ inline cplx cadd(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
__device__ __host__ inline cplx cscale(cplx a, double s) { return {a.re * s, a.im * s}; }
__device__ __host__ inline cplx cconj(cplx a) { return {a.re, -a.im}; }

}  // namespace lt
