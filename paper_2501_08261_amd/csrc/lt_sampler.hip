// On-device parallel-tempered ensemble sampler (hot-path step a11).
//
// Per step: for each half of every temperature's ensemble, a Goodman-Weare
// stretch proposal Y = X_j + z (X_k - X_j) against a random walker j of the
// other half, z ~ g(z) on [1/a, a] with g ~ 1/sqrt(z); uniform-box prior;
// batched logL of all proposals; Metropolis-Hastings with
// log alpha = (d - 1) ln z + beta_T (logL_Y - logL_X) + (logP_Y - logP_X);
// then adjacent-temperature swaps (hottest pair first) between walker k at
// beta_i and walker (k + r) mod W at beta_{i+1}, accepted with
// min(1, exp((beta_i - beta_{i+1}) (logL_{i+1} - logL_i))).
// Random numbers: Philox4x32-10 (Salmon et al. 2011), key = seed, counter =
// (step, purpose, slot, 0), uniforms (u + 1/2) 2^-32.  One step is captured
// once as a HIP graph and replayed.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/lisatd.h"
#include "lt_rng.hpp"

namespace lt_s {

using namespace lt_rng;

constexpr int kMaxDim = 32;

struct Dev {
  int T, W, d, kind, target, n_gauss;
  double a, t_c;
  uint32_t k0, k1;
  double *X, *logl, *logp, *beta;
  double *Y, *ylogl, *ylogp, *ylogz, *yu;
  double* params;           // [T*W][16] (set_state) / [T*W/2][16] (proposals)
  double *lo, *hi, *gmean, *gicov;
  uint64_t* step;
  int64_t *acc, *prop, *sacc, *sprop;
  // flow move on the cold rung (beta_0 = 1)
  double *fy, *fqy, *fqx, *fylogl, *fylogp;
  int64_t *facc, *fprop;
  // symmetry fold of the flow move: coordinate fold_i (-1: none) is mapped into the window
  // [fold_c0, fold_c0 + fold_p) before the flow sees it; a proposal takes one of the copies
  // y + k fold_p inside the prior range, uniformly
  int fold_i;
  double fold_p, fold_c0;
  double *fxf, *flkx;       // folded cold positions [W][d]; log(number of copies) of each
  double walk;              // > 0: the flow move is a random walk of this step in the flow's latent space
  double p_flow;            // probability that a step runs the flow move (1: every step)
  int* fgate;               // this step's draw: 1 = the flow move runs
  int fexcl;                // 1: a step that runs the flow move skips the cold rung's stretch moves
  // mixture of two flows (second flow attached): component weights w1, 1 - w1; the second
  // flow's proposals and log densities
  double mw1;
  double *fy2, *fqy2, *fqx2;
};

__device__ inline void to_params(const Dev& D, const double* x, double* p) {
  for (int i = 0; i < 16; ++i) p[i] = 0.0;
  p[0] = x[0];
  p[1] = x[1];
  if (D.kind == LT_PARAMS_PRECESSING14) {
    double s1, c1, s2, c2;
    sincos(x[3], &s1, &c1);
    sincos(x[4], &s2, &c2);
    p[2] = x[2] * s1 * c2; p[3] = x[2] * s1 * s2; p[4] = x[2] * c1;
    sincos(x[6], &s1, &c1);
    sincos(x[7], &s2, &c2);
    p[5] = x[5] * s1 * c2; p[6] = x[5] * s1 * s2; p[7] = x[5] * c1;
    p[8] = x[8]; p[9] = x[9]; p[10] = x[10]; p[13] = x[11]; p[12] = x[12]; p[14] = x[13];
  } else {
    p[4] = x[2]; p[7] = x[3];
    p[8] = x[4]; p[9] = x[5]; p[10] = x[6]; p[13] = x[7]; p[12] = x[8]; p[14] = x[9];
  }
  p[11] = D.t_c;
}

__device__ inline double log_prior(const Dev& D, const double* x) {
  for (int i = 0; i < D.d; ++i)
    if (!(x[i] >= D.lo[i] && x[i] <= D.hi[i])) return -INFINITY;
  return 0.0;
}

// proposals for half h: one thread per (temperature, walker of the half).  excl: on a step
// whose gate runs the flow move, the cold rung proposes nothing (unphysical parameter rows,
// which the likelihood skips after its per-template setup)
__global__ void k_propose(Dev D, int h, int excl) {
  const int half = D.W / 2;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= D.T * half) return;
  const int t = idx / half, kk = idx - t * half;
  if (excl && t == 0 && *D.fgate) {
    D.ylogp[idx] = -INFINITY;
    if (D.target == LT_TARGET_TDI)
      for (int i = 0; i < 16; ++i) D.params[(int64_t)idx * 16 + i] = 0.0;
    return;
  }
  const int k = h * half + kk;
  uint32_t c[4] = {(uint32_t)*D.step, kTagMove + (uint32_t)h, (uint32_t)(t * D.W + k), 0u};
  philox4x32_10(c, D.k0, D.k1);
  int jj = (int)(u01(c[0]) * half);
  jj = jj < half ? jj : half - 1;
  const int j = (1 - h) * half + jj;
  const double zr = (D.a - 1.0) * u01(c[1]) + 1.0;
  const double z = zr * zr / D.a;
  const double* xk = D.X + ((int64_t)t * D.W + k) * D.d;
  const double* xj = D.X + ((int64_t)t * D.W + j) * D.d;
  double* y = D.Y + (int64_t)idx * D.d;
  for (int i = 0; i < D.d; ++i) y[i] = xj[i] + z * (xk[i] - xj[i]);
  D.ylogz[idx] = log(z);
  D.yu[idx] = u01(c[2]);
  D.ylogp[idx] = log_prior(D, y);
  if (D.target == LT_TARGET_TDI) to_params(D, y, D.params + (int64_t)idx * 16);
}

// all walkers (set_state): prior and parameter rows
__global__ void k_prepare_all(Dev D) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= D.T * D.W) return;
  const double* x = D.X + (int64_t)idx * D.d;
  D.logp[idx] = log_prior(D, x);
  if (D.target == LT_TARGET_TDI) to_params(D, x, D.params + (int64_t)idx * 16);
}

// analytic test target: log of an equal-weight mixture of Gaussians
__global__ void k_gauss(Dev D, const double* xs, int64_t count, double* out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= count) return;
  const double* x = xs + idx * D.d;
  double best = -INFINITY, q[2];
  for (int m = 0; m < D.n_gauss; ++m) {
    double dx[kMaxDim];
    for (int i = 0; i < D.d; ++i) dx[i] = x[i] - D.gmean[m * D.d + i];
    double s = 0.0;
    for (int i = 0; i < D.d; ++i) {
      double r = 0.0;
      for (int j = 0; j < D.d; ++j) r += D.gicov[i * D.d + j] * dx[j];
      s += dx[i] * r;
    }
    q[m] = -0.5 * s;
    best = fmax(best, q[m]);
  }
  double acc = 0.0;
  for (int m = 0; m < D.n_gauss; ++m) acc += exp(q[m] - best);
  out[idx] = best + log(acc / D.n_gauss);
}

__global__ void k_accept(Dev D, int h, int excl) {
  const int half = D.W / 2;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= D.T * half) return;
  const int t = idx / half, kk = idx - t * half;
  if (excl && t == 0 && *D.fgate) return;   // no cold stretch move on this step: nothing counted
  const int64_t w = (int64_t)t * D.W + h * half + kk;
  const double lly = D.ylogl[idx], lpy = D.ylogp[idx];
  const double la = (D.d - 1) * D.ylogz[idx] + D.beta[t] * (lly - D.logl[w]) + (lpy - D.logp[w]);
  const bool ok = lpy > -INFINITY && !isnan(lly) && lly > -INFINITY && log(D.yu[idx]) < la;
  if (ok) {
    const double* y = D.Y + (int64_t)idx * D.d;
    double* x = D.X + w * D.d;
    for (int i = 0; i < D.d; ++i) x[i] = y[i];
    D.logl[w] = lly;
    D.logp[w] = lpy;
  }
  D.acc[w] += ok ? 1 : 0;
  D.prop[w] += 1;
}

// flow proposals y (one per cold walker): prior and parameter rows
// copies v + k P of a folded value v inside [lo, hi]: k in [k_min, k_min + n)
__device__ inline int fold_copies(double v, double P, double lo, double hi, double* k_min) {
  const double a = ceil((lo - v) / P), b = floor((hi - v) / P);
  *k_min = a;
  return b >= a ? (int)(b - a) + 1 : 0;
}

// cold positions folded for the flow, and log(number of copies) of each
__global__ void k_flow_fold(Dev D) {
#pragma clang fp contract(off)
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= D.W) return;
  const double* x = D.X + (int64_t)k * D.d;
  double* xf = D.fxf + (int64_t)k * D.d;
  for (int i = 0; i < D.d; ++i) xf[i] = x[i];
  double lk = 0.0;
  if (D.fold_i >= 0) {
    const int i = D.fold_i;
    const double v = D.fold_c0 + ((x[i] - D.fold_c0) - D.fold_p * floor((x[i] - D.fold_c0) / D.fold_p));
    xf[i] = v;
    double km;
    const int n = fold_copies(v, D.fold_p, D.lo[i], D.hi[i], &km);
    lk = n > 0 ? log((double)n) : 0.0;
  }
  D.flkx[k] = lk;
}

// mixture proposal: walker k takes the second flow's point when u >= w1, u from counter
// (step, 0x900, k, 0) (both flows mapped the same base normals)
__global__ void k_flow_pick(Dev D) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= D.W || !*D.fgate) return;
  uint32_t c[4] = {(uint32_t)*D.step, kTagFlowM, (uint32_t)k, 0u};
  philox4x32_10(c, D.k0, D.k1);
  if (!(u01(c[0]) < D.mw1))
    for (int i = 0; i < D.d; ++i) D.fy[(int64_t)k * D.d + i] = D.fy2[(int64_t)k * D.d + i];
}

// log(w1 q1 + w2 q2) into a, from the two flows' log densities a (first) and b (second)
__device__ inline double log_mix(double a, double b, double lw1, double lw2) {
  const double x = lw1 + a, y = lw2 + b;
  if (x == y) return x + 0.69314718055994530942;
  return x > y ? x + log1p(exp(y - x)) : y + log1p(exp(x - y));
}

__global__ void k_flow_mixq(Dev D) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= D.W || !*D.fgate) return;
  const double lw1 = log(D.mw1), lw2 = log1p(-D.mw1);
  D.fqy[k] = log_mix(D.fqy[k], D.fqy2[k], lw1, lw2);
  D.fqx[k] = log_mix(D.fqx[k], D.fqx2[k], lw1, lw2);
}

// whether this step runs the flow move: u < p_flow, u from counter (step, 0x800, 0, 0)
__global__ void k_flow_gate(Dev D) {
  uint32_t c[4] = {(uint32_t)*D.step, kTagFlowG, 0u, 0u};
  philox4x32_10(c, D.k0, D.k1);
  *D.fgate = u01(c[0]) < D.p_flow ? 1 : 0;
}

// proposals: unfolded into a uniformly drawn copy (log q(y) less log(number of copies)), prior,
// likelihood parameters.  A step without the flow move gets unphysical parameter rows (zero
// masses), which the likelihood skips after its per-template setup.
__global__ void k_flow_prep(Dev D) {
#pragma clang fp contract(off)
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= D.W) return;
  double* y = D.fy + (int64_t)k * D.d;
  if (!*D.fgate) {
    D.fylogp[k] = -INFINITY;
    if (D.target == LT_TARGET_TDI)
      for (int i = 0; i < 16; ++i) D.params[(int64_t)k * 16 + i] = 0.0;
    return;
  }
  bool out = false;
  if (D.fold_i >= 0) {
    const int i = D.fold_i;
    const double v = y[i];
    double km;
    const int n = (v >= D.fold_c0 && v < D.fold_c0 + D.fold_p) ? fold_copies(v, D.fold_p, D.lo[i], D.hi[i], &km) : 0;
    if (n > 0) {
      uint32_t c[4] = {(uint32_t)*D.step, kTagFlowC, (uint32_t)k, 0u};
      philox4x32_10(c, D.k0, D.k1);
      int j = (int)(u01(c[0]) * (double)n);
      j = j < n - 1 ? j : n - 1;
      y[i] = v + (km + (double)j) * D.fold_p;
      D.fqy[k] -= log((double)n);
    } else {
      out = true;      // outside the fold window: no copy of it is proposed
    }
  }
  D.fylogp[k] = out ? -INFINITY : log_prior(D, y);
  if (D.target == LT_TARGET_TDI) to_params(D, y, D.params + (int64_t)k * 16);
}

// independence Metropolis-Hastings with the flow density q:
// log alpha = beta_0 (logL_y - logL_x) + (logP_y - logP_x) + log q(x) - log q(y)
__global__ void k_flow_accept(Dev D) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= D.W || !*D.fgate) return;
  uint32_t c[4] = {(uint32_t)*D.step, kTagFlowU, (uint32_t)k, 0u};
  philox4x32_10(c, D.k0, D.k1);
  const double lly = D.fylogl[k], lpy = D.fylogp[k];
  const double la = D.beta[0] * (lly - D.logl[k]) + (lpy - D.logp[k]) + ((D.fqx[k] - D.flkx[k]) - D.fqy[k]);
  const bool ok = lpy > -INFINITY && !isnan(lly) && lly > -INFINITY && !isnan(la) && log(u01(c[0])) < la;
  if (ok) {
    const double* y = D.fy + (int64_t)k * D.d;
    double* x = D.X + (int64_t)k * D.d;
    for (int i = 0; i < D.d; ++i) x[i] = y[i];
    D.logl[k] = lly;
    D.logp[k] = lpy;
  }
  D.facc[k] += ok ? 1 : 0;
  D.fprop[k] += 1;
}

// tempering swaps, hottest adjacent pair first; one workgroup, then the step counter advances
__global__ void k_swap(Dev D) {
  const uint64_t step = *D.step;
  for (int i = D.T - 2; i >= 0; --i) {
    uint32_t c[4] = {(uint32_t)step, kTagShift + (uint32_t)i, 0u, 0u};
    philox4x32_10(c, D.k0, D.k1);
    const int r = (int)(c[0] % (uint32_t)D.W);
    const double db = D.beta[i] - D.beta[i + 1];
    for (int k = threadIdx.x; k < D.W; k += blockDim.x) {
      const int k2 = (k + r) % D.W;
      const int64_t a = (int64_t)i * D.W + k, b = (int64_t)(i + 1) * D.W + k2;
      uint32_t e[4] = {(uint32_t)step, kTagSwap + (uint32_t)i, (uint32_t)k, 0u};
      philox4x32_10(e, D.k0, D.k1);
      const double la = db * (D.logl[b] - D.logl[a]);
      const bool ok = log(u01(e[0])) < la;
      if (ok) {
        for (int q = 0; q < D.d; ++q) {
          double tmp = D.X[a * D.d + q];
          D.X[a * D.d + q] = D.X[b * D.d + q];
          D.X[b * D.d + q] = tmp;
        }
        double tl = D.logl[a]; D.logl[a] = D.logl[b]; D.logl[b] = tl;
        double tp = D.logp[a]; D.logp[a] = D.logp[b]; D.logp[b] = tp;
      }
      D.sacc[a] += ok ? 1 : 0;
      D.sprop[a] += 1;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *D.step = step + 1;
}

}  // namespace lt_s

using namespace lt_s;

namespace lt {
void set_error(const std::string& msg);   // thread-local message returned by lt_last_error()
int flow_dim(const lt_flow* f);
int flow_max_batch(const lt_flow* f);
int flow_device(const lt_flow* f);
hipError_t flow_propose(lt_flow* f, int n, const uint64_t* step, uint32_t k0, uint32_t k1, double* y, double* logq_y,
                        hipStream_t st, const int* gate);
hipError_t flow_logq(lt_flow* f, const double* x, int n, double* logq, hipStream_t st, const int* gate);
hipError_t flow_propose_logq(lt_flow* f, int n, const uint64_t* step, uint32_t k0, uint32_t k1, double* y,
                             double* logq_y, const double* x, double* logq_x, hipStream_t st, const int* gate);
hipError_t flow_walk(lt_flow* f, const double* x, int n, const uint64_t* step, uint32_t k0, uint32_t k1, double sigma,
                     double* y, double* lq_y, double* lq_x, hipStream_t st, const int* gate);
}

struct lt_sampler {
  int device = 0;
  lt_sampler_cfg cfg{};
  lt_wf_cfg wf{};
  lt_grid grid{};
  lt_orbit orbit{};
  std::vector<double> orbit_pos, orbit_ltt;   // owned copy of a table orbit's arrays
  lt_tdi_cfg tdi{};
  lt_psd psd{};
  lt_data data{};
  lt_ctx* ctx = nullptr;
  Dev D{};
  std::vector<void*> allocs;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  lt_flow* flow = nullptr;
  lt_flow* flow2 = nullptr;    // second component of a mixture proposal (nullable)
  void* ws = nullptr;          // likelihood workspace (TDI target), sized for the whole ensemble
  size_t ws_bytes = 0;
};

#define S_HIP(call)                                                                  \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess) {                                                          \
      lt::set_error(std::string(#call) + ": " + hipGetErrorString(e_));             \
      return LT_ERR_DEVICE;                                                          \
    }                                                                                \
  } while (0)

template <typename T>
static lt_status salloc(lt_sampler* s, T** p, size_t count) {
  void* q = nullptr;
  S_HIP(hipMalloc(&q, count * sizeof(T) + 64));
  s->allocs.push_back(q);
  *p = (T*)q;
  return LT_OK;
}

static lt_status sfail(lt_status st, const char* msg) {
  lt::set_error(msg);
  return st;
}

// logL of `count` parameter rows / coordinates on the capture or default stream
static lt_status eval_logl(lt_sampler* s, const double* xs, int64_t count, double* out, hipStream_t st) {
  if (s->cfg.target == LT_TARGET_GAUSS) {
    hipLaunchKernelGGL(k_gauss, dim3((unsigned)((count + 127) / 128)), dim3(128), 0, st, s->D, xs, count, out);
    S_HIP(hipGetLastError());
    return LT_OK;
  }
  lt_status r = lt_tdi_loglike(s->ctx, s->D.params, count, &s->wf, &s->grid, &s->orbit, &s->tdi, &s->psd, &s->data,
                               out, nullptr, nullptr, s->ws, s->ws_bytes, st);
  if (r != LT_OK) lt::set_error(std::string("logL: ") + lt_last_error());
  return r;
}

static lt_status record_step(lt_sampler* s, hipStream_t st) {
  const int half = s->cfg.n_walkers / 2;
  const int n = s->cfg.n_temps * half;
  const bool flow = s->flow && s->D.p_flow > 0.0;
  const int excl = flow && s->D.fexcl ? 1 : 0;
  if (flow) {
    // the step's draw of the flow move, read by the stretch half-steps when excl is set
    hipLaunchKernelGGL(k_flow_gate, dim3(1), dim3(1), 0, st, s->D);
    S_HIP(hipGetLastError());
  }
  for (int h = 0; h < 2; ++h) {
    hipLaunchKernelGGL(k_propose, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, st, s->D, h, excl);
    S_HIP(hipGetLastError());
    lt_status r = eval_logl(s, s->D.Y, n, s->D.ylogl, st);
    if (r != LT_OK) return r;
    hipLaunchKernelGGL(k_accept, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, st, s->D, h, excl);
    S_HIP(hipGetLastError());
  }
  if (flow) {
    const int W = s->cfg.n_walkers;
    hipLaunchKernelGGL(k_flow_fold, dim3((unsigned)((W + 127) / 128)), dim3(128), 0, st, s->D);
    S_HIP(hipGetLastError());
    if (s->D.walk > 0.0) {
      // y = f^-1(f(x) + walk eps): fqx, fqy carry log q - log N of the two latent points
      S_HIP(lt::flow_walk(s->flow, s->D.fxf, W, s->D.step, s->D.k0, s->D.k1, s->D.walk, s->D.fy, s->D.fqy, s->D.fqx,
                          st, s->D.fgate));
    } else if (s->flow2) {
      // mixture: both flows map the step's base normals, each walker keeps its component's
      // point, and the mixture density is taken at the proposals and the current positions
      const unsigned gw = (unsigned)((W + 127) / 128);
      S_HIP(lt::flow_propose(s->flow, W, s->D.step, s->D.k0, s->D.k1, s->D.fy, s->D.fqy, st, s->D.fgate));
      S_HIP(lt::flow_propose(s->flow2, W, s->D.step, s->D.k0, s->D.k1, s->D.fy2, s->D.fqy2, st, s->D.fgate));
      hipLaunchKernelGGL(k_flow_pick, dim3(gw), dim3(128), 0, st, s->D);
      S_HIP(hipGetLastError());
      S_HIP(lt::flow_logq(s->flow, s->D.fy, W, s->D.fqy, st, s->D.fgate));
      S_HIP(lt::flow_logq(s->flow2, s->D.fy, W, s->D.fqy2, st, s->D.fgate));
      S_HIP(lt::flow_logq(s->flow, s->D.fxf, W, s->D.fqx, st, s->D.fgate));
      S_HIP(lt::flow_logq(s->flow2, s->D.fxf, W, s->D.fqx2, st, s->D.fgate));
      hipLaunchKernelGGL(k_flow_mixq, dim3(gw), dim3(128), 0, st, s->D);
      S_HIP(hipGetLastError());
    } else {
      // the flow's kernels return at once in a step that the gate leaves without the move
      S_HIP(lt::flow_propose_logq(s->flow, W, s->D.step, s->D.k0, s->D.k1, s->D.fy, s->D.fqy, s->D.fxf, s->D.fqx, st,
                                  s->D.fgate));
    }
    hipLaunchKernelGGL(k_flow_prep, dim3((unsigned)((W + 127) / 128)), dim3(128), 0, st, s->D);
    S_HIP(hipGetLastError());
    lt_status r = eval_logl(s, s->D.fy, W, s->D.fylogl, st);
    if (r != LT_OK) return r;
    hipLaunchKernelGGL(k_flow_accept, dim3((unsigned)((W + 127) / 128)), dim3(128), 0, st, s->D);
    S_HIP(hipGetLastError());
  }
  const int nt = s->cfg.n_walkers < 1024 ? s->cfg.n_walkers : 1024;
  hipLaunchKernelGGL(k_swap, dim3(1), dim3((unsigned)((nt + 63) / 64 * 64)), 0, st, s->D);
  S_HIP(hipGetLastError());
  return LT_OK;
}

extern "C" {

lt_status lt_sampler_create(int hip_device, const lt_sampler_cfg* cfg, const lt_wf_cfg* wf, const lt_grid* grid,
                            const lt_orbit* orbit, const lt_tdi_cfg* tdi, const lt_psd* psd, const lt_data* data,
                            lt_sampler** out) {
  if (!cfg || !out || !cfg->lo || !cfg->hi) return sfail(LT_ERR_NULL, "null sampler argument");
  if (cfg->n_walkers < 4 || cfg->n_walkers % 2 || cfg->n_walkers > 65536) return sfail(LT_ERR_SHAPE, "n_walkers");
  if (cfg->n_temps < 1 || cfg->n_temps > 64) return sfail(LT_ERR_SHAPE, "n_temps");
  if (cfg->dim < 1 || cfg->dim > kMaxDim) return sfail(LT_ERR_SHAPE, "dim");
  if (!(cfg->stretch_a > 1.0) || !(cfg->t_max >= 1.0)) return sfail(LT_ERR_CONFIG, "stretch_a > 1, t_max >= 1");
  if (cfg->target == LT_TARGET_TDI) {
    if (!wf || !grid || !orbit || !tdi || !psd || !data) return sfail(LT_ERR_NULL, "TDI target needs the likelihood");
    int need = cfg->param_kind == LT_PARAMS_PRECESSING14 ? 14 : (cfg->param_kind == LT_PARAMS_ALIGNED10 ? 10 : -1);
    if (need != cfg->dim) return sfail(LT_ERR_CONFIG, "param_kind does not match dim");
    if ((int64_t)cfg->n_temps * cfg->n_walkers > 65535) return sfail(LT_ERR_SHAPE, "too many walkers for one batch");
  } else if (cfg->target == LT_TARGET_GAUSS) {
    if (!cfg->gauss_mean || !cfg->gauss_icov || cfg->n_gauss < 1 || cfg->n_gauss > 2)
      return sfail(LT_ERR_CONFIG, "Gaussian target needs 1 or 2 means and an inverse covariance");
  } else {
    return sfail(LT_ERR_CONFIG, "target");
  }
  S_HIP(hipSetDevice(hip_device));
  lt_sampler* s = new lt_sampler();
  s->device = hip_device;
  s->cfg = *cfg;
  if (cfg->target == LT_TARGET_TDI) {
    s->wf = *wf; s->grid = *grid; s->orbit = *orbit; s->tdi = *tdi; s->psd = *psd; s->data = *data;
    if (orbit->kind == LT_ORBIT_TABLE && orbit->pos && orbit->ltt && orbit->n_tab > 0) {
      s->orbit_pos.assign(orbit->pos, orbit->pos + orbit->n_tab * 9);
      s->orbit_ltt.assign(orbit->ltt, orbit->ltt + orbit->n_tab * 6);
      s->orbit.pos = s->orbit_pos.data();
      s->orbit.ltt = s->orbit_ltt.data();
    }
    if (lt_ctx_create(hip_device, &s->ctx) != LT_OK) {
      delete s;
      return sfail(LT_ERR_DEVICE, "context");
    }
  }
  const int T = cfg->n_temps, W = cfg->n_walkers, d = cfg->dim;
  Dev& D = s->D;
  D.T = T; D.W = W; D.d = d; D.kind = cfg->param_kind; D.target = cfg->target; D.n_gauss = cfg->n_gauss;
  D.a = cfg->stretch_a; D.t_c = cfg->t_c;
  D.fold_i = -1;
  D.walk = 0.0;
  D.p_flow = 1.0;
  D.fexcl = 0;
  D.mw1 = 1.0;
  D.fold_p = 1.0;
  D.fold_c0 = 0.0;
  D.k0 = (uint32_t)(cfg->seed & 0xffffffffu);
  D.k1 = (uint32_t)(cfg->seed >> 32);
  lt_status r = LT_OK;
  const size_t TW = (size_t)T * W;
  if ((r = salloc(s, &D.X, TW * d)) || (r = salloc(s, &D.logl, TW)) || (r = salloc(s, &D.logp, TW)) ||
      (r = salloc(s, &D.beta, T)) || (r = salloc(s, &D.Y, TW / 2 * d)) || (r = salloc(s, &D.ylogl, TW / 2)) ||
      (r = salloc(s, &D.ylogp, TW / 2)) || (r = salloc(s, &D.ylogz, TW / 2)) || (r = salloc(s, &D.yu, TW / 2)) ||
      (r = salloc(s, &D.params, TW * 16)) || (r = salloc(s, &D.lo, d)) || (r = salloc(s, &D.hi, d)) ||
      (r = salloc(s, &D.gmean, 2 * d)) || (r = salloc(s, &D.gicov, (size_t)d * d)) || (r = salloc(s, &D.step, 1)) ||
      (r = salloc(s, &D.acc, TW)) || (r = salloc(s, &D.prop, TW)) || (r = salloc(s, &D.sacc, TW)) ||
      (r = salloc(s, &D.sprop, TW)) || (r = salloc(s, &D.fy, (size_t)W * d)) || (r = salloc(s, &D.fqy, W)) ||
      (r = salloc(s, &D.fqx, W)) || (r = salloc(s, &D.fylogl, W)) || (r = salloc(s, &D.fylogp, W)) ||
      (r = salloc(s, &D.facc, W)) || (r = salloc(s, &D.fprop, W)) || (r = salloc(s, &D.fxf, (size_t)W * d)) ||
      (r = salloc(s, &D.flkx, W)) || (r = salloc(s, &D.fgate, 1)) || (r = salloc(s, &D.fy2, (size_t)W * d)) ||
      (r = salloc(s, &D.fqy2, W)) || (r = salloc(s, &D.fqx2, W))) {
    lt_sampler_destroy(s);
    return r;
  }
  std::vector<double> beta(T);
  for (int i = 0; i < T; ++i) beta[i] = T > 1 ? std::pow(cfg->t_max, -(double)i / (double)(T - 1)) : 1.0;
  S_HIP(hipMemcpy(D.beta, beta.data(), T * sizeof(double), hipMemcpyHostToDevice));
  S_HIP(hipMemcpy(D.lo, cfg->lo, d * sizeof(double), hipMemcpyHostToDevice));
  S_HIP(hipMemcpy(D.hi, cfg->hi, d * sizeof(double), hipMemcpyHostToDevice));
  if (cfg->target == LT_TARGET_GAUSS) {
    S_HIP(hipMemcpy(D.gmean, cfg->gauss_mean, (size_t)cfg->n_gauss * d * sizeof(double), hipMemcpyHostToDevice));
    S_HIP(hipMemcpy(D.gicov, cfg->gauss_icov, (size_t)d * d * sizeof(double), hipMemcpyHostToDevice));
  } else {
    // chunks of templates: on short grids larger than the default 256, which cuts the fixed
    // costs of each chunk, while a chunk's residual (3 n samples per template) stays within
    // 128 MiB, so that the FFT passes find it in the last-level cache after the response kernel
    // wrote it (2^14 samples: 512 templates; 256 from 2^16 samples up), and its workspace
    // within 4 GiB
    lt_tuning tu;
    lt_status r2 = lt_ctx_get_tuning(s->ctx, &tu);
    const size_t rsz = s->wf.precision == LT_FP64 ? 8 : 4;
    for (int ch = tu.chunk * 2; r2 == LT_OK && ch <= 4096 && ch / 2 < (int)TW; ch *= 2) {
      if ((size_t)ch * 3 * (size_t)s->grid.n * rsz > ((size_t)128 << 20)) break;
      size_t b = 0;
      lt_tuning t2 = tu;
      t2.chunk = ch;
      if ((r2 = lt_ctx_set_tuning(s->ctx, &t2)) != LT_OK) break;
      if ((r2 = lt_workspace_size(s->ctx, TW, &s->wf, &s->grid, &s->tdi, &b, nullptr)) != LT_OK) break;
      if (b > ((size_t)4 << 30)) break;
      tu.chunk = ch;
    }
    if (r2 == LT_OK) r2 = lt_ctx_set_tuning(s->ctx, &tu);
    // one workspace for every likelihood call of the sampler (at most the whole ensemble per
    // call), so that a captured step allocates nothing
    size_t wsb = 0;
    if (r2 == LT_OK) r2 = lt_workspace_size(s->ctx, TW, &s->wf, &s->grid, &s->tdi, &wsb, nullptr);
    if (r2 == LT_OK) r2 = salloc(s, (unsigned char**)&s->ws, wsb);
    if (r2 != LT_OK) {
      lt_sampler_destroy(s);
      return r2;
    }
    s->ws_bytes = wsb;
  }
  S_HIP(hipStreamCreateWithFlags(&s->cap, hipStreamNonBlocking));
  s->cfg.lo = s->cfg.hi = s->cfg.gauss_mean = s->cfg.gauss_icov = nullptr;
  *out = s;
  return LT_OK;
}

lt_status lt_sampler_destroy(lt_sampler* s) {
  if (!s) return sfail(LT_ERR_NULL, "null sampler");
  (void)hipSetDevice(s->device);
  (void)hipDeviceSynchronize();
  if (s->exec) (void)hipGraphExecDestroy(s->exec);
  if (s->graph) (void)hipGraphDestroy(s->graph);
  if (s->cap) (void)hipStreamDestroy(s->cap);
  for (void* p : s->allocs) (void)hipFree(p);
  if (s->ctx) lt_ctx_destroy(s->ctx);
  delete s;
  return LT_OK;
}

lt_status lt_sampler_set_state(lt_sampler* s, const double* pos) {
  if (!s || !pos) return sfail(LT_ERR_NULL, "null argument");
  S_HIP(hipSetDevice(s->device));
  const int64_t TW = (int64_t)s->cfg.n_temps * s->cfg.n_walkers;
  S_HIP(hipMemcpy(s->D.X, pos, TW * s->cfg.dim * sizeof(double), hipMemcpyHostToDevice));
  hipLaunchKernelGGL(k_prepare_all, dim3((unsigned)((TW + 127) / 128)), dim3(128), 0, s->cap, s->D);
  S_HIP(hipGetLastError());
  lt_status r = eval_logl(s, s->D.X, TW, s->D.logl, s->cap);
  if (r != LT_OK) return r;
  std::vector<int64_t> z(TW, 0);
  uint64_t zero = 0;
  S_HIP(hipMemcpyAsync(s->D.step, &zero, sizeof(uint64_t), hipMemcpyHostToDevice, s->cap));
  for (int64_t* p : {s->D.acc, s->D.prop, s->D.sacc, s->D.sprop})
    S_HIP(hipMemcpyAsync(p, z.data(), TW * sizeof(int64_t), hipMemcpyHostToDevice, s->cap));
  for (int64_t* p : {s->D.facc, s->D.fprop})
    S_HIP(hipMemcpyAsync(p, z.data(), s->cfg.n_walkers * sizeof(int64_t), hipMemcpyHostToDevice, s->cap));
  S_HIP(hipStreamSynchronize(s->cap));
  return LT_OK;
}

lt_status lt_sampler_step(lt_sampler* s, int n_steps, void* stream) {
  if (!s) return sfail(LT_ERR_NULL, "null sampler");
  if (n_steps < 0) return sfail(LT_ERR_SHAPE, "n_steps");
  S_HIP(hipSetDevice(s->device));
  if (!s->exec) {
    S_HIP(hipStreamSynchronize(s->cap));
    S_HIP(hipStreamBeginCapture(s->cap, hipStreamCaptureModeThreadLocal));
    lt_status r = record_step(s, s->cap);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s->cap, &g);
    if (r != LT_OK) {
      if (g) (void)hipGraphDestroy(g);
      return r;
    }
    S_HIP(e);
    s->graph = g;
    S_HIP(hipGraphInstantiate(&s->exec, s->graph, nullptr, nullptr, 0));
  }
  for (int i = 0; i < n_steps; ++i) S_HIP(hipGraphLaunch(s->exec, (hipStream_t)stream));
  return LT_OK;
}

lt_status lt_sampler_get_state(lt_sampler* s, double* pos, double* logl, double* logp, uint64_t* step,
                               int64_t* counters) {
  if (!s) return sfail(LT_ERR_NULL, "null sampler");
  S_HIP(hipSetDevice(s->device));
  S_HIP(hipDeviceSynchronize());
  const int64_t TW = (int64_t)s->cfg.n_temps * s->cfg.n_walkers;
  if (pos) S_HIP(hipMemcpy(pos, s->D.X, TW * s->cfg.dim * sizeof(double), hipMemcpyDeviceToHost));
  if (logl) S_HIP(hipMemcpy(logl, s->D.logl, TW * sizeof(double), hipMemcpyDeviceToHost));
  if (logp) S_HIP(hipMemcpy(logp, s->D.logp, TW * sizeof(double), hipMemcpyDeviceToHost));
  if (step) S_HIP(hipMemcpy(step, s->D.step, sizeof(uint64_t), hipMemcpyDeviceToHost));
  if (counters) {
    std::vector<int64_t> v(TW);
    int64_t* src[4] = {s->D.acc, s->D.prop, s->D.sacc, s->D.sprop};
    for (int q = 0; q < 4; ++q) {
      S_HIP(hipMemcpy(v.data(), src[q], TW * sizeof(int64_t), hipMemcpyDeviceToHost));
      int64_t t = 0;
      for (int64_t x : v) t += x;
      counters[q] = t;
    }
  }
  return LT_OK;
}

lt_status lt_sampler_set_flow(lt_sampler* s, lt_flow* flow) {
  if (!s) return sfail(LT_ERR_NULL, "null sampler");
  if (flow) {
    if (lt::flow_dim(flow) != s->cfg.dim) return sfail(LT_ERR_CONFIG, "flow dimension differs from the sampler's");
    if (lt::flow_max_batch(flow) < s->cfg.n_walkers) return sfail(LT_ERR_SHAPE, "flow max_batch < n_walkers");
    if (lt::flow_device(flow) != s->device) return sfail(LT_ERR_CONFIG, "flow lives on another device");
  }
  S_HIP(hipSetDevice(s->device));
  S_HIP(hipDeviceSynchronize());
  if (s->exec) (void)hipGraphExecDestroy(s->exec);
  if (s->graph) (void)hipGraphDestroy(s->graph);
  s->exec = nullptr;
  s->graph = nullptr;
  s->flow = flow;
  return LT_OK;
}

lt_status lt_sampler_set_flow_mixture(lt_sampler* s, lt_flow* second, double w_first) {
  if (!s) return sfail(LT_ERR_NULL, "null sampler");
  if (second) {
    if (!(w_first > 0.0 && w_first < 1.0)) return sfail(LT_ERR_CONFIG, "w_first must lie in (0, 1)");
    if (lt::flow_dim(second) != s->cfg.dim) return sfail(LT_ERR_CONFIG, "flow dimension differs from the sampler's");
    if (lt::flow_max_batch(second) < s->cfg.n_walkers) return sfail(LT_ERR_SHAPE, "flow max_batch < n_walkers");
    if (lt::flow_device(second) != s->device) return sfail(LT_ERR_CONFIG, "flow lives on another device");
    if (s->D.walk > 0.0) return sfail(LT_ERR_CONFIG, "the latent walk takes one flow");
  }
  S_HIP(hipSetDevice(s->device));
  S_HIP(hipDeviceSynchronize());
  if (s->exec) (void)hipGraphExecDestroy(s->exec);
  if (s->graph) (void)hipGraphDestroy(s->graph);
  s->exec = nullptr;
  s->graph = nullptr;
  s->flow2 = second;
  s->D.mw1 = second ? w_first : 1.0;
  return LT_OK;
}

lt_status lt_sampler_set_flow_fold(lt_sampler* s, int index, double period, double start) {
  if (!s) return sfail(LT_ERR_NULL, "null sampler");
  if (index < -1 || index >= s->cfg.dim) return sfail(LT_ERR_CONFIG, "fold index");
  if (index >= 0 && !(period > 0.0 && std::isfinite(period) && std::isfinite(start)))
    return sfail(LT_ERR_CONFIG, "fold period must be positive and finite, start finite");
  S_HIP(hipSetDevice(s->device));
  S_HIP(hipDeviceSynchronize());
  if (s->exec) (void)hipGraphExecDestroy(s->exec);
  if (s->graph) (void)hipGraphDestroy(s->graph);
  s->exec = nullptr;
  s->graph = nullptr;
  s->D.fold_i = index;
  s->D.fold_p = index >= 0 ? period : 1.0;
  s->D.fold_c0 = index >= 0 ? start : 0.0;
  return LT_OK;
}

lt_status lt_sampler_set_flow_walk(lt_sampler* s, double step) {
  if (!s) return sfail(LT_ERR_NULL, "null sampler");
  if (!(step >= 0.0 && std::isfinite(step))) return sfail(LT_ERR_CONFIG, "walk step must be finite and >= 0");
  if (step > 0.0 && s->flow2) return sfail(LT_ERR_CONFIG, "the latent walk takes one flow (a mixture is attached)");
  S_HIP(hipSetDevice(s->device));
  S_HIP(hipDeviceSynchronize());
  if (s->exec) (void)hipGraphExecDestroy(s->exec);
  if (s->graph) (void)hipGraphDestroy(s->graph);
  s->exec = nullptr;
  s->graph = nullptr;
  s->D.walk = step;
  return LT_OK;
}

lt_status lt_flow_set_mix(lt_sampler* s, double p_flow) {
  if (!s) return sfail(LT_ERR_NULL, "null sampler");
  if (!(p_flow >= 0.0 && p_flow <= 1.0)) return sfail(LT_ERR_CONFIG, "p_flow must lie in [0, 1]");
  S_HIP(hipSetDevice(s->device));
  S_HIP(hipDeviceSynchronize());
  if (s->exec) (void)hipGraphExecDestroy(s->exec);
  if (s->graph) (void)hipGraphDestroy(s->graph);
  s->exec = nullptr;
  s->graph = nullptr;
  s->D.p_flow = p_flow;
  return LT_OK;
}

lt_status lt_sampler_set_flow_exclusive(lt_sampler* s, int on) {
  if (!s) return sfail(LT_ERR_NULL, "null sampler");
  if (on != 0 && on != 1) return sfail(LT_ERR_CONFIG, "exclusive must be 0 or 1");
  S_HIP(hipSetDevice(s->device));
  S_HIP(hipDeviceSynchronize());
  if (s->exec) (void)hipGraphExecDestroy(s->exec);
  if (s->graph) (void)hipGraphDestroy(s->graph);
  s->exec = nullptr;
  s->graph = nullptr;
  s->D.fexcl = on;
  return LT_OK;
}

lt_status lt_sampler_flow_counts(lt_sampler* s, int64_t* counts) {
  if (!s || !counts) return sfail(LT_ERR_NULL, "null argument");
  S_HIP(hipSetDevice(s->device));
  S_HIP(hipDeviceSynchronize());
  const int W = s->cfg.n_walkers;
  std::vector<int64_t> v(W);
  int64_t* src[2] = {s->D.facc, s->D.fprop};
  for (int q = 0; q < 2; ++q) {
    S_HIP(hipMemcpy(v.data(), src[q], W * sizeof(int64_t), hipMemcpyDeviceToHost));
    int64_t t = 0;
    for (int64_t x : v) t += x;
    counts[q] = t;
  }
  return LT_OK;
}

}  // extern "C"
