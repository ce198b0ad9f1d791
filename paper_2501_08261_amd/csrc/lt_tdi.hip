// Per-template setup, mode / polarisation kernels, and the fused TDI response
// kernel (hot-path steps a1-a8 of the time-domain LISA likelihood).
#include "lt_kernels.hpp"
#include "lt_wave.hpp"

namespace lt {

constexpr int kNT = 256;      // threads per workgroup
constexpr int kTile = 1024;   // output samples per workgroup of the TDI kernel

int tdi_tile() { return kTile; }

// ------------------------------------------------------------------ setup
__global__ __launch_bounds__(64) void k_setup(const double* params, int64_t batch, double f_low, double f_ref,
                                              GridDev g, TplConst* tc, int32_t* status) {
  int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  TplConst c;
  int ok = setup_template(params + 16 * b, f_low, f_ref, g.t0, g.dt, c);
  tc[b] = c;
  if (status) status[b] = ok ? 0 : 1;
}

hipError_t launch_setup(const double* params, int64_t batch, double f_low, double f_ref, GridDev g,
                        TplConst* tc, int32_t* status, hipStream_t s) {
  dim3 grid((unsigned)((batch + 63) / 64));
  hipLaunchKernelGGL(k_setup, grid, dim3(64), 0, s, params, batch, f_low, f_ref, g, tc, status);
  return hipGetLastError();
}

// ------------------------------------------------------------------ modes
__global__ __launch_bounds__(kNT) void k_modes(const TplConst* tc, int mode_mask, GridDev g, double* modes) {
  int64_t n = (int64_t)blockIdx.x * kNT + threadIdx.x;
  int b = blockIdx.y;
  if (n >= g.n) return;
  const TplConst& c = tc[b];
  cplx h[5] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}};
  if (c.valid != 0.0) cp_modes_fp64(c, g.t0 + (double)n * g.dt, h);
  int nm = __popc(mode_mask);
  int j = 0;
  for (int i = 0; i < 5; ++i) {
    if (!(mode_mask & (1 << i))) continue;
    double* dst = modes + 2 * (((int64_t)b * nm + j) * g.n + n);
    dst[0] = h[i].re;
    dst[1] = h[i].im;
    ++j;
  }
}

hipError_t launch_modes(const TplConst* tc, int64_t batch, int mode_mask, GridDev g, double* modes, hipStream_t s) {
  dim3 grid((unsigned)((g.n + kNT - 1) / kNT), (unsigned)batch);
  hipLaunchKernelGGL(k_modes, grid, dim3(kNT), 0, s, tc, mode_mask, g, modes);
  return hipGetLastError();
}

// Polarisations h+, hx on the grid (steps a2-a4), one thread per sample:
// h[b][0][n] = h+, h[b][1][n] = hx in the storage type R.
template <typename R, bool PREC>
__global__ __launch_bounds__(kNT) void k_wave(const TplConst* tc, int mode_mask, GridDev g, R* h) {
  int64_t n = (int64_t)blockIdx.x * kNT + threadIdx.x;
  int b = blockIdx.y;
  if (n >= g.n) return;
  const TplConst& c = tc[b];
  cx<R> v{(R)0, (R)0};
  if (c.valid != 0.0 && (double)n >= c.n_start - 1.0) v = polarization_t<R, PREC>(c, mode_mask, g.t0 + (double)n * g.dt);
  h[(2 * (int64_t)b) * g.n + n] = v.re;
  h[(2 * (int64_t)b + 1) * g.n + n] = -v.im;
}

template <typename R>
static hipError_t launch_wave_t(const TplConst* tc, int64_t batch, int mode_mask, int precessing, GridDev g, R* h,
                                hipStream_t s) {
  dim3 grid((unsigned)((g.n + kNT - 1) / kNT), (unsigned)batch);
  if (precessing)
    hipLaunchKernelGGL((k_wave<R, true>), grid, dim3(kNT), 0, s, tc, mode_mask, g, h);
  else
    hipLaunchKernelGGL((k_wave<R, false>), grid, dim3(kNT), 0, s, tc, mode_mask, g, h);
  return hipGetLastError();
}

hipError_t launch_polarizations(const TplConst* tc, int64_t batch, int mode_mask, int precessing, GridDev g,
                                double* hpc, hipStream_t s) {
  return launch_wave_t<double>(tc, batch, mode_mask, precessing, g, hpc, s);
}

hipError_t launch_wave(const TplConst* tc, int64_t batch, int mode_mask, int precessing, int precision, GridDev g,
                       void* h, hipStream_t s) {
  if (precision == 0) return launch_wave_t<double>(tc, batch, mode_mask, precessing, g, (double*)h, s);
  return launch_wave_t<float>(tc, batch, mode_mask, precessing, g, (float*)h, s);
}

// ------------------------------------------------------- Lagrange weights
// Centred K-tap Lagrange weights for fraction f in [0, 1): nodes at offsets
// o_i = i - K/2 + 1, w_i = prod_{j != i} (f - o_j) / (o_i - o_j), computed
// with prefix / suffix products (no division by f - o_j).
template <int K>
struct LagDen {
  double inv[K];
  __host__ __device__ constexpr LagDen() : inv() {
    for (int i = 0; i < K; ++i) {
      double p = 1.0;
      for (int j = 0; j < K; ++j)
        if (j != i) p *= (double)(i - j);
      inv[i] = 1.0 / p;
    }
  }
};

template <typename R, int K>
__device__ inline void lag_weights(R f, R* w) {
  constexpr LagDen<K> den;
  R d[K];
#pragma unroll
  for (int j = 0; j < K; ++j) d[j] = f - (R)(j - K / 2 + 1);
  R pre = (R)1;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    w[i] = pre;
    pre *= d[i];
  }
  R suf = (R)1;
#pragma unroll
  for (int i = K - 1; i >= 0; --i) {
    w[i] *= suf * (R)den.inv[i];
    suf *= d[i];
  }
}

// Stencil start for fractional index s: the K taps are a[j0 - K/2 + 1 .. j0 + K/2].
// Windows are sized so that every stencil lies inside; the clamp only keeps
// memory accesses in bounds and never triggers for valid inputs.
template <int K>
__device__ inline int stencil_start(double fl, int len) {
  int j = (int)fl - K / 2 + 1;
  j = j < 0 ? 0 : j;
  return j > len - K ? len - K : j;
}

// One series at fractional index s, in the product form
//   sum_i c_i y_i prod_{j != i} d_j,  d_j = f - o_j,  c_i = 1 / prod_{j != i}(o_i - o_j),
// accumulated left to right: S_i = S_{i-1} d_i + c_i y_i P_{i-1}, P_i = P_{i-1} d_i.
template <typename R, int K>
__device__ inline R lag1(const R* a, int len, double s) {
  constexpr LagDen<K> den;
  double fl = floor(s);
  const R f = (R)(s - fl);
  const R* p = a + stencil_start<K>(fl, len);
  R P = f - (R)(-K / 2 + 1);
  R S = (R)den.inv[0] * p[0];
#pragma unroll
  for (int i = 1; i < K; ++i) {
    const R d = f - (R)(i - K / 2 + 1);
    S = S * d + (R)den.inv[i] * p[i] * P;
    P *= d;
  }
  return S;
}

// Two series sharing one set of weights (h+ and hx at the same time).
template <typename R, int K>
__device__ inline void lag2(const R* a, const R* b, int len, double s, R& ra, R& rb) {
  double fl = floor(s);
  R w[K];
  lag_weights<R, K>((R)(s - fl), w);
  const int j = stencil_start<K>(fl, len);
  const R* pa = a + j;
  const R* pb = b + j;
  R acc_a = (R)0, acc_b = (R)0;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    acc_a += w[i] * pa[i];
    acc_b += w[i] * pb[i];
  }
  ra = acc_a;
  rb = acc_b;
}

__device__ inline int64_t floordiv(int64_t a, int64_t b) {
  int64_t q = a / b;
  return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

// four-point (cubic) Lagrange weights at x in [0,1) for nodes -1, 0, 1, 2
__device__ inline void cubic_w(double x, double* w) {
  double xm1 = x - 1.0, xm2 = x - 2.0, xp1 = x + 1.0;
  w[0] = -x * xm1 * xm2 * (1.0 / 6.0);
  w[1] = xp1 * xm1 * xm2 * 0.5;
  w[2] = -xp1 * x * xm2 * 0.5;
  w[3] = xp1 * x * xm1 * (1.0 / 6.0);
}

// per node: for each link (P+, Px, D_s, L), then D_r for each spacecraft
constexpr int kNL = 4;
constexpr int kNodeVals = 6 * kNL + 3;
__constant__ int kRecv[6] = {1, 2, 0, 2, 0, 1};     // receiver spacecraft (0-based) of links 1,2,3,-1,-2,-3
__constant__ int kRecvLink[3] = {2, 0, 1};          // a link received by spacecraft 1, 2, 3

// ------------------------------------------------------- fused TDI kernel
// One workgroup = one template x one tile of kTile output samples.
//  B: per-link geometry at the orbit nodes covering the tile (LDS, FP64)
//  A: h+, hx on the window of grid samples the six links read (LDS)
//  C: y_slr for the tile plus the TDI halos; h is interpolated with K taps at
//     the three receiver times and the six sender times (LDS)
//  D: X, Y, Z from y interpolated at the TDI delays, then A, E, T (global)
template <typename R, int K>
__global__ __launch_bounds__(kNT) void k_tdi(TdiLaunch P, int HY, int WMAX, int NNMAX) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ long long s_w0;
  __shared__ int s_W, s_skip;
  const int tid = threadIdx.x;
  const int b = blockIdx.y;
  const int64_t N = P.g.n;
  const int64_t n0 = (int64_t)blockIdx.x * kTile;
  const TplConst& c = P.tc[b];
  // y is needed on [n0 - HY, n0 + kTile + K/2]: the centred stencils of the
  // shortest TDI delays reach K/2 - 1 samples past the last output sample
  const int MY = kTile + HY + K / 2 + 1;
  R* yb = (R*)smem;
  R* hpb = yb + 6 * MY;
  R* hxb = hpb + WMAX;
  double* nd = (double*)(smem + (((size_t)(6 * MY + 2 * WMAX) * sizeof(R) + 15) & ~(size_t)15));
  const double inv_dt = P.g.inv_dt;
  const int64_t m_lo = n0 - HY, m_hi = m_lo + MY - 1;
  const int S = P.orb.spacing;
  const int64_t jn_lo = floordiv(m_lo, S) - 1 + P.orb.j0;
  const int64_t jn_hi = floordiv(m_hi, S) + 2 + P.orb.j0;
  const int NN = (int)(jn_hi - jn_lo + 1);

  // B: node geometry
  for (int i = tid; i < NN * 9; i += kNT) {
    int nl = i / 9, q = i - nl * 9;
    double* o = nd + nl * kNodeVals;
    if (q < 6) {
      const double* e = P.orb.tab + (jn_lo + nl) * kNodeStride + q * kNodeLink;
      double un = c.u[0] * e[7] + c.u[1] * e[8] + c.u[2] * e[9];
      double vn = c.v[0] * e[7] + c.v[1] * e[8] + c.v[2] * e[9];
      double kn = c.k[0] * e[7] + c.k[1] * e[8] + c.k[2] * e[9];
      double inv = 1.0 / (1.0 - kn);
      o[q * kNL + 0] = 0.5 * (un * un - vn * vn) * inv;
      o[q * kNL + 1] = un * vn * inv;
      o[q * kNL + 2] = e[0] + (c.k[0] * e[4] + c.k[1] * e[5] + c.k[2] * e[6]);
      o[q * kNL + 3] = e[0];
    } else {
      const double* e = P.orb.tab + (jn_lo + nl) * kNodeStride + kRecvLink[q - 6] * kNodeLink;
      o[6 * kNL + (q - 6)] = c.k[0] * e[1] + c.k[1] * e[2] + c.k[2] * e[3];
    }
  }
  __syncthreads();
  if (tid == 0) {
    double dmin = 1e300, dmax = -1e300;
    for (int i = 0; i < NN; ++i) {
      const double* o = nd + i * kNodeVals;
      for (int q = 0; q < 6; ++q) { dmin = fmin(dmin, o[q * kNL + 2]); dmax = fmax(dmax, o[q * kNL + 2]); }
      for (int q = 0; q < 3; ++q) { dmin = fmin(dmin, o[6 * kNL + q]); dmax = fmax(dmax, o[6 * kNL + q]); }
    }
    long long w0 = (long long)m_lo - (long long)ceil(dmax * inv_dt) - K / 2 - 2;
    long long w1 = (long long)m_hi - (long long)floor(dmin * inv_dt) + K / 2 + 2;
    int W = (int)(w1 - w0 + 1);
    int bad = 0;
    if (W > WMAX) { W = WMAX; bad = 1; }
    s_w0 = w0;
    s_W = W;
    // every needed h sample precedes the f_low start (or the template is invalid): all zero
    s_skip = (c.valid == 0.0 || (double)w1 < c.n_start - 2.0) ? 1 : 0;
    if (bad && P.status) P.status[b] = 3;
  }
  __syncthreads();
  const long long w0 = s_w0;
  const int W = s_W;
  const int skip = s_skip;

  if (!skip) {
    // A: polarisations of the window from the waveform buffer
    const R* hg = (const R*)P.h + (2 * (int64_t)b) * N;
    for (int i = tid; i < W; i += kNT) {
      long long j = w0 + i;
      bool in = j >= 0 && j < N;
      hpb[i] = in ? hg[j] : (R)0;
      hxb[i] = in ? hg[N + j] : (R)0;
    }
    __syncthreads();
    // C: link responses y_slr for m in [m_lo, m_hi]
    for (int mi = tid; mi < MY; mi += kNT) {
      int64_t m = m_lo + mi;
      if (m < 0 || m >= N) {
#pragma unroll
        for (int li = 0; li < 6; ++li) yb[li * MY + mi] = (R)0;
        continue;
      }
      int64_t q = floordiv(m, S);
      int jl = (int)(q + P.orb.j0 - jn_lo);
      double w[4];
      cubic_w((double)(m - q * S) / (double)S, w);
      const double* o0 = nd + (jl - 1) * kNodeVals;
      const double mloc = (double)(m - w0);
      R hpr[3], hxr[3];
#pragma unroll
      for (int sc = 0; sc < 3; ++sc) {
        double Dr = 0.0;
#pragma unroll
        for (int r = 0; r < 4; ++r) Dr += w[r] * o0[r * kNodeVals + 6 * kNL + sc];
        lag2<R, K>(hpb, hxb, W, mloc - Dr * inv_dt, hpr[sc], hxr[sc]);
      }
#pragma unroll
      for (int li = 0; li < 6; ++li) {
        double v0 = 0.0, v1 = 0.0, v2 = 0.0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double* o = o0 + r * kNodeVals + li * kNL;
          v0 += w[r] * o[0];
          v1 += w[r] * o[1];
          v2 += w[r] * o[2];
        }
        R hps, hxs;
        lag2<R, K>(hpb, hxb, W, mloc - v2 * inv_dt, hps, hxs);
        const int rc = kRecv[li];
        yb[li * MY + mi] = (R)v0 * (hps - hpr[rc]) + (R)v1 * (hxs - hxr[rc]);
      }
    }
    __syncthreads();
  }
  // D: TDI and A, E, T
  const R* data = (const R*)P.data;
  R* out = (R*)P.out;
  for (int ni = tid; ni < kTile; ni += kNT) {
    int64_t n = n0 + ni;
    if (n >= N) break;
    R ch[3] = {(R)0, (R)0, (R)0};
    if (!skip) {
      int64_t q = floordiv(n, S);
      int jl = (int)(q + P.orb.j0 - jn_lo);
      double w[4];
      cubic_w((double)(n - q * S) / (double)S, w);
      double Lt[6];
#pragma unroll
      for (int li = 0; li < 6; ++li) {
        double a = 0.0;
#pragma unroll
        for (int r = 0; r < 4; ++r) a += w[r] * nd[(jl - 1 + r) * kNodeVals + li * kNL + 3];
        Lt[li] = a;
      }
      for (int cc = 0; cc < 3; ++cc) {
        R acc = (R)0;
        for (int t = 0; t < P.terms.n_terms[cc]; ++t) {
          const Term& tm = P.terms.t[cc][t];
          double D = 0.0;
          for (int k = 0; k < tm.nd; ++k) D += (double)tm.dcnt[k] * Lt[tm.dlink[k]];
          double s = (double)(n - m_lo) - D * inv_dt;
          R yv = lag1<R, K>(yb + tm.link * MY, MY, s);
          acc += tm.sign > 0 ? yv : -yv;
        }
        ch[cc] = acc;
      }
    }
    R o0, o1, o2;
    if (P.out_mode == 1) {
      o0 = ch[0]; o1 = ch[1]; o2 = ch[2];
    } else {
      const R r2 = (R)0.70710678118654752440, r6 = (R)0.40824829046386301637, r3 = (R)0.57735026918962576451;
      o0 = (ch[2] - ch[0]) * r2;
      o1 = (ch[0] - (R)2 * ch[1] + ch[2]) * r6;
      o2 = (ch[0] + ch[1] + ch[2]) * r3;
      if (P.out_mode == 2) {
        o0 -= data[n];
        o1 -= data[N + n];
        o2 -= data[2 * N + n];
      }
    }
    int64_t base = (int64_t)b * 3 * N + n;
    out[base] = o0;
    out[base + N] = o1;
    out[base + 2 * N] = o2;
  }
}

template <typename R, int K>
static hipError_t launch_tdi_t(const TdiLaunch& P, hipStream_t s) {
  int HY = (int)ceil(7.0 * P.orb.max_light_time * P.g.inv_dt * 1.001) + K / 2 + 2;
  int spread = (int)ceil(2.0 * P.orb.max_light_time * P.g.inv_dt * 1.01) + 8;
  const int MY = kTile + HY + K / 2 + 1;
  int WMAX = MY + spread + K + 8;
  int NNMAX = MY / P.orb.spacing + 5;
  if (HY + 8 > P.orb.spacing || K / 2 + 9 > P.orb.spacing) return hipErrorInvalidValue;   // node table covers one spacing of halo
  size_t bytes = (((size_t)(6 * MY + 2 * WMAX) * sizeof(R) + 15) & ~(size_t)15) +
                 (size_t)NNMAX * kNodeVals * sizeof(double);
  if (bytes > 160 * 1024) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute((const void*)k_tdi<R, K>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)bytes);
  if (e != hipSuccess) return e;
  dim3 grid((unsigned)((P.g.n + kTile - 1) / kTile), (unsigned)P.batch);
  hipLaunchKernelGGL((k_tdi<R, K>), grid, dim3(kNT), bytes, s, P, HY, WMAX, NNMAX);
  return hipGetLastError();
}

template <typename R>
static hipError_t launch_tdi_k(const TdiLaunch& P, hipStream_t s) {
  switch (P.taps) {
    case 2: return launch_tdi_t<R, 2>(P, s);
    case 4: return launch_tdi_t<R, 4>(P, s);
    case 6: return launch_tdi_t<R, 6>(P, s);
    case 8: return launch_tdi_t<R, 8>(P, s);
    case 12: return launch_tdi_t<R, 12>(P, s);
    case 16: return launch_tdi_t<R, 16>(P, s);
    case 24: return launch_tdi_t<R, 24>(P, s);
    case 32: return launch_tdi_t<R, 32>(P, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_tdi(const TdiLaunch& P, hipStream_t s) {
  return P.precision == 0 ? launch_tdi_k<double>(P, s) : launch_tdi_k<float>(P, s);
}

}  // namespace lt
