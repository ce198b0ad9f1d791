// Fisher matrix and Fisher-initialised starting points for the sampler.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "../../include/lisatd.h"
#include "lt_rng.hpp"

namespace lt {
void set_error(const std::string& msg);
}

namespace {

lt_status ferr(lt_status s, const std::string& m) {
  lt::set_error(m);
  return s;
}

#define F_HIP(call)                                                                  \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess) return ferr(LT_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// sampling coordinates -> 16-entry parameter row (layout of include/lisatd.h)
void to_params_host(const double* x, int kind, double t_c, double* p) {
  for (int i = 0; i < 16; ++i) p[i] = 0.0;
  p[0] = x[0];
  p[1] = x[1];
  if (kind == LT_PARAMS_PRECESSING14) {
    p[2] = x[2] * std::sin(x[3]) * std::cos(x[4]);
    p[3] = x[2] * std::sin(x[3]) * std::sin(x[4]);
    p[4] = x[2] * std::cos(x[3]);
    p[5] = x[5] * std::sin(x[6]) * std::cos(x[7]);
    p[6] = x[5] * std::sin(x[6]) * std::sin(x[7]);
    p[7] = x[5] * std::cos(x[6]);
    p[8] = x[8]; p[9] = x[9]; p[10] = x[10]; p[13] = x[11]; p[12] = x[12]; p[14] = x[13];
  } else {
    p[4] = x[2]; p[7] = x[3];
    p[8] = x[4]; p[9] = x[5]; p[10] = x[6]; p[13] = x[7]; p[12] = x[8]; p[14] = x[9];
  }
  p[11] = t_c;
}

// D[i] = (h[2i] - h[2i+1]) / (2 eps_i); S[(i,j)] = D_i + D_j (i <= j, row-major upper triangle)
__global__ void k_fd(const double* h, int64_t len, int d, const double* inv2eps, double* D) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int i = blockIdx.y;
  if (k >= len) return;
  D[i * len + k] = (h[(2 * (int64_t)i) * len + k] - h[(2 * (int64_t)i + 1) * len + k]) * inv2eps[i];
}

__global__ void k_pairs(const double* D, int64_t len, int d, double* S) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int q = blockIdx.y;
  if (k >= len) return;
  int i = 0, rem = q;
  while (rem >= d - i) { rem -= d - i; ++i; }
  int j = i + rem;
  S[q * len + k] = D[i * len + k] + D[j * len + k];
}

// Jacobi eigen-decomposition of a symmetric matrix (a destroyed; v = eigenvectors in columns)
void jacobi(std::vector<double>& a, int n, std::vector<double>& w, std::vector<double>& v) {
  v.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) v[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += a[p * n + q] * a[p * n + q];
    if (off < 1e-30) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = a[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        double theta = (a[q * n + q] - a[p * n + p]) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {
          double akp = a[k * n + p], akq = a[k * n + q];
          a[k * n + p] = c * akp - s * akq;
          a[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          double apk = a[p * n + k], aqk = a[q * n + k];
          a[p * n + k] = c * apk - s * aqk;
          a[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double vkp = v[k * n + p], vkq = v[k * n + q];
          v[k * n + p] = c * vkp - s * vkq;
          v[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = a[i * n + i];
}


}  // namespace

extern "C" {

lt_status lt_fisher(lt_ctx* ctx, const double* x0, int param_kind, double t_c, const double* steps,
                    const lt_wf_cfg* cfg, const lt_grid* grid, const lt_orbit* orbit, const lt_tdi_cfg* tdi,
                    const lt_psd* psd, double* gamma) {
  if (!ctx || !x0 || !steps || !cfg || !grid || !orbit || !tdi || !psd || !gamma)
    return ferr(LT_ERR_NULL, "null argument");
  const int d = param_kind == LT_PARAMS_PRECESSING14 ? 14 : (param_kind == LT_PARAMS_ALIGNED10 ? 10 : -1);
  if (d < 0) return ferr(LT_ERR_CONFIG, "param_kind must be ALIGNED10 or PRECESSING14");
  if (cfg->precision != LT_FP64) return ferr(LT_ERR_CONFIG, "the Fisher matrix is computed in FP64");
  for (int i = 0; i < d; ++i)
    if (!(steps[i] > 0.0)) return ferr(LT_ERR_CONFIG, "steps must be positive");
  const int64_t n = grid->n, len = 3 * n;
  std::vector<double> rows((size_t)2 * d * 16), x(d);
  for (int i = 0; i < d; ++i)
    for (int sgn = 0; sgn < 2; ++sgn) {
      for (int k = 0; k < d; ++k) x[k] = x0[k];
      x[i] += sgn == 0 ? steps[i] : -steps[i];
      to_params_host(x.data(), param_kind, t_c, rows.data() + (2 * i + sgn) * 16);
    }
  const int npair = d * (d + 1) / 2;
  double *dp = nullptr, *dh = nullptr, *dD = nullptr, *dS = nullptr, *dinv = nullptr, *dout = nullptr;
  lt_status st = LT_OK;
  auto cleanup = [&]() {
    for (double* q : {dp, dh, dD, dS, dinv, dout})
      if (q) (void)hipFree(q);
  };
  std::vector<double> inv(d);
  for (int i = 0; i < d; ++i) inv[i] = 0.5 / steps[i];
  if (hipMalloc(&dp, rows.size() * sizeof(double)) != hipSuccess ||
      hipMalloc(&dh, (size_t)2 * d * len * sizeof(double)) != hipSuccess ||
      hipMalloc(&dD, (size_t)d * len * sizeof(double)) != hipSuccess ||
      hipMalloc(&dS, (size_t)npair * len * sizeof(double)) != hipSuccess ||
      hipMalloc(&dinv, d * sizeof(double)) != hipSuccess || hipMalloc(&dout, npair * sizeof(double)) != hipSuccess) {
    cleanup();
    return ferr(LT_ERR_DEVICE, "Fisher scratch allocation failed");
  }
  std::vector<double> nij(npair);
  do {
    if (hipMemcpy(dp, rows.data(), rows.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dinv, inv.data(), d * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
      st = ferr(LT_ERR_DEVICE, "copy");
      break;
    }
    lt_tdi_cfg t = *tdi;
    t.out_xyz = 0;
    if ((st = lt_lisa_tdi_response(ctx, dp, 2 * d, cfg, grid, orbit, &t, dh, nullptr, nullptr))) break;
    hipLaunchKernelGGL(k_fd, dim3((unsigned)((len + 255) / 256), d), dim3(256), 0, 0, dh, len, d, dinv, dD);
    hipLaunchKernelGGL(k_pairs, dim3((unsigned)((len + 255) / 256), npair), dim3(256), 0, 0, dD, len, d, dS);
    if (hipGetLastError() != hipSuccess) {
      st = ferr(LT_ERR_DEVICE, "finite-difference kernels");
      break;
    }
    if ((st = lt_noise_inner(ctx, dS, npair, grid, psd, tdi->channels, LT_FP64, dout, nullptr))) break;
    if (hipMemcpy(nij.data(), dout, npair * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
      st = ferr(LT_ERR_DEVICE, "copy back");
      break;
    }
  } while (false);
  cleanup();
  if (st) return st;
  // (D_i + D_j | D_i + D_j) = G_ii + 2 G_ij + G_jj, and (2 D_i | 2 D_i) = 4 G_ii
  std::vector<double> diag(d);
  int q = 0;
  std::vector<int> qi(npair), qj(npair);
  for (int i = 0; i < d; ++i)
    for (int j = i; j < d; ++j, ++q) { qi[q] = i; qj[q] = j; }
  for (q = 0; q < npair; ++q)
    if (qi[q] == qj[q]) diag[qi[q]] = 0.25 * nij[q];
  for (q = 0; q < npair; ++q) {
    int i = qi[q], j = qj[q];
    double g = (i == j) ? diag[i] : 0.5 * (nij[q] - diag[i] - diag[j]);
    gamma[i * d + j] = g;
    gamma[j * d + i] = g;
  }
  return LT_OK;
}

lt_status lt_fisher_draw(const double* x0, const double* gamma, int dim, const double* lo, const double* hi,
                         int64_t count, uint64_t seed, double reg, double* out) {
  if (!x0 || !gamma || !lo || !hi || !out) return ferr(LT_ERR_NULL, "null argument");
  if (dim < 1 || dim > 64 || count < 0) return ferr(LT_ERR_SHAPE, "dim / count");
  if (!(reg >= 0.0)) return ferr(LT_ERR_CONFIG, "reg must be >= 0");
  // The eigen floor is applied to D Gamma D with D = diag(Gamma_ii^-1/2): in that unit-diagonal basis
  // the floor is relative to the best-measured combination of comparably scaled coordinates, so a
  // parameter measured in large units (mass, distance) is not flattened by one measured in small ones.
  std::vector<double> a((size_t)dim * dim), w, v, dg(dim);
  for (int i = 0; i < dim; ++i) dg[i] = gamma[i * dim + i] > 0.0 ? std::sqrt(gamma[i * dim + i]) : 1.0;
  for (int i = 0; i < dim; ++i)
    for (int j = 0; j < dim; ++j)
      a[i * dim + j] = 0.5 * (gamma[i * dim + j] + gamma[j * dim + i]) / (dg[i] * dg[j]);
  jacobi(a, dim, w, v);
  double wmax = 0.0;
  for (double x : w) wmax = std::fmax(wmax, x);
  if (!(wmax > 0.0)) return ferr(LT_ERR_CONFIG, "Fisher matrix has no positive eigenvalue");
  std::vector<double> sd(dim);
  for (int i = 0; i < dim; ++i) sd[i] = 1.0 / std::sqrt(std::fmax(w[i], reg * wmax));
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  std::vector<double> z(dim);
  for (int64_t s = 0; s < count; ++s) {
    double* o = out + s * dim;
    bool inside = false;
    for (int attempt = 0; attempt < 64 && !inside; ++attempt) {
      for (int i = 0; i < dim; i += 2) {
        uint32_t c[4] = {(uint32_t)s, (uint32_t)attempt, (uint32_t)i, 0x51u};
        lt_rng::philox4x32_10(c, k0, k1);
        double u1 = ((double)c[0] + 0.5) * 2.3283064365386963e-10, u2 = ((double)c[1] + 0.5) * 2.3283064365386963e-10;
        double r = std::sqrt(-2.0 * std::log(u1));
        z[i] = r * std::cos(2.0 * M_PI * u2);
        if (i + 1 < dim) z[i + 1] = r * std::sin(2.0 * M_PI * u2);
      }
      inside = true;
      for (int i = 0; i < dim; ++i) {
        double acc = x0[i];
        double y = 0.0;
        for (int k = 0; k < dim; ++k) y += v[i * dim + k] * sd[k] * z[k];
        acc += y / dg[i];
        o[i] = acc;
        if (!(acc >= lo[i] && acc <= hi[i])) inside = false;
      }
    }
    for (int i = 0; i < dim; ++i) o[i] = std::fmin(hi[i], std::fmax(lo[i], o[i]));
  }
  return LT_OK;
}

}  // extern "C"
