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
  Orb o;
  if (c.valid != 0.0 && orbital_state(c, g.t0 + (double)n * g.dt, o)) cp_modes5(c, o, h);
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

template <bool PREC>
__global__ __launch_bounds__(kNT) void k_pol(const TplConst* tc, int mode_mask, GridDev g, double* hpc) {
  int64_t n = (int64_t)blockIdx.x * kNT + threadIdx.x;
  int b = blockIdx.y;
  if (n >= g.n) return;
  const TplConst& c = tc[b];
  cplx h{0.0, 0.0};
  if (c.valid != 0.0) h = polarization<PREC>(c, mode_mask, g.t0 + (double)n * g.dt);
  hpc[(2 * (int64_t)b) * g.n + n] = h.re;
  hpc[(2 * (int64_t)b + 1) * g.n + n] = -h.im;
}

hipError_t launch_polarizations(const TplConst* tc, int64_t batch, int mode_mask, int precessing, GridDev g,
                                double* hpc, hipStream_t s) {
  dim3 grid((unsigned)((g.n + kNT - 1) / kNT), (unsigned)batch);
  if (precessing)
    hipLaunchKernelGGL(k_pol<true>, grid, dim3(kNT), 0, s, tc, mode_mask, g, hpc);
  else
    hipLaunchKernelGGL(k_pol<false>, grid, dim3(kNT), 0, s, tc, mode_mask, g, hpc);
  return hipGetLastError();
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

// Interpolate array a[0..len) (zero outside) at fractional index s.
template <typename R, int K>
__device__ inline R lag1(const R* a, int len, double s) {
  double fl = floor(s);
  int j0 = (int)fl;
  R w[K];
  lag_weights<R, K>((R)(s - fl), w);
  R acc = (R)0;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    int idx = j0 - K / 2 + 1 + i;
    idx = idx < 0 ? 0 : (idx >= len ? len - 1 : idx);   // memory safety only: windows are sized to contain every stencil
    acc += w[i] * a[idx];
  }
  return acc;
}

template <typename R, int K>
__device__ inline void lag2(const R* a, const R* b, int len, double s, R& ra, R& rb) {
  double fl = floor(s);
  int j0 = (int)fl;
  R w[K];
  lag_weights<R, K>((R)(s - fl), w);
  R acc_a = (R)0, acc_b = (R)0;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    int idx = j0 - K / 2 + 1 + i;
    idx = idx < 0 ? 0 : (idx >= len ? len - 1 : idx);
    acc_a += w[i] * a[idx];
    acc_b += w[i] * b[idx];
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

constexpr int kND = 5;   // per node and link: P+, Px, D_s, D_r, L

// ------------------------------------------------------- fused TDI kernel
// One workgroup = one template x one tile of kTile output samples.
//  B: per-link geometry at the orbit nodes covering the tile (LDS, FP64)
//  A: h+, hx on the window of grid samples the six links read (LDS)
//  C: y_slr for the tile plus the TDI halo, h interpolated with K taps (LDS)
//  D: X, Y, Z from y interpolated at the TDI delays, then A, E, T (global)
template <typename R, int K, bool PREC>
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
  for (int i = tid; i < NN * 6; i += kNT) {
    int nl = i / 6, li = i % 6;
    const double* e = P.orb.tab + (jn_lo + nl) * kNodeStride + li * kNodeLink;
    double L = e[0];
    double un = c.u[0] * e[7] + c.u[1] * e[8] + c.u[2] * e[9];
    double vn = c.v[0] * e[7] + c.v[1] * e[8] + c.v[2] * e[9];
    double kn = c.k[0] * e[7] + c.k[1] * e[8] + c.k[2] * e[9];
    double inv = 1.0 / (1.0 - kn);
    double* o = nd + (nl * 6 + li) * kND;
    o[0] = 0.5 * (un * un - vn * vn) * inv;
    o[1] = un * vn * inv;
    o[2] = L + (c.k[0] * e[4] + c.k[1] * e[5] + c.k[2] * e[6]);
    o[3] = c.k[0] * e[1] + c.k[1] * e[2] + c.k[2] * e[3];
    o[4] = L;
  }
  __syncthreads();
  if (tid == 0) {
    double dmin = 1e300, dmax = -1e300;
    for (int i = 0; i < NN * 6; ++i) {
      dmin = fmin(dmin, fmin(nd[i * kND + 2], nd[i * kND + 3]));
      dmax = fmax(dmax, fmax(nd[i * kND + 2], nd[i * kND + 3]));
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
    // A: polarisations on the window
    for (int i = tid; i < W; i += kNT) {
      long long j = w0 + i;
      R hp = (R)0, hx = (R)0;
      if (j >= 0 && j < N) {
        cplx h = polarization<PREC>(c, P.mode_mask, P.g.t0 + (double)j * P.g.dt);
        hp = (R)h.re;
        hx = (R)(-h.im);
      }
      hpb[i] = hp;
      hxb[i] = hx;
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
#pragma unroll
      for (int li = 0; li < 6; ++li) {
        double v[4] = {0, 0, 0, 0};
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double* o = nd + ((jl - 1 + r) * 6 + li) * kND;
#pragma unroll
          for (int e = 0; e < 4; ++e) v[e] += w[r] * o[e];
        }
        double ss = (double)(m - w0) - v[2] * inv_dt;
        double sr = (double)(m - w0) - v[3] * inv_dt;
        R hps, hxs, hpr, hxr;
        lag2<R, K>(hpb, hxb, W, ss, hps, hxs);
        lag2<R, K>(hpb, hxb, W, sr, hpr, hxr);
        yb[li * MY + mi] = (R)v[0] * (hps - hpr) + (R)v[1] * (hxs - hxr);
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
        for (int r = 0; r < 4; ++r) a += w[r] * nd[((jl - 1 + r) * 6 + li) * kND + 4];
        Lt[li] = a;
      }
      for (int cc = 0; cc < 3; ++cc) {
        R acc = (R)0;
        for (int t = 0; t < P.terms.n_terms[cc]; ++t) {
          const Term& tm = P.terms.t[cc][t];
          double D = 0.0;
#pragma unroll
          for (int li = 0; li < 6; ++li) D += (double)tm.cnt[li] * Lt[li];
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

template <typename R, int K, bool PREC>
static hipError_t launch_tdi_t(const TdiLaunch& P, hipStream_t s) {
  int HY = (int)ceil(7.0 * P.orb.max_light_time * P.g.inv_dt * 1.001) + K / 2 + 2;
  int spread = (int)ceil(2.0 * P.orb.max_light_time * P.g.inv_dt * 1.01) + 8;
  const int MY = kTile + HY + K / 2 + 1;
  int WMAX = MY + spread + K + 8;
  int NNMAX = MY / P.orb.spacing + 5;
  if (HY + 8 > P.orb.spacing || K / 2 + 9 > P.orb.spacing) return hipErrorInvalidValue;   // node table covers one spacing of halo
  size_t bytes = (((size_t)(6 * MY + 2 * WMAX) * sizeof(R) + 15) & ~(size_t)15) +
                 (size_t)NNMAX * 6 * kND * sizeof(double);
  if (bytes > 160 * 1024) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute((const void*)k_tdi<R, K, PREC>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)bytes);
  if (e != hipSuccess) return e;
  dim3 grid((unsigned)((P.g.n + kTile - 1) / kTile), (unsigned)P.batch);
  hipLaunchKernelGGL((k_tdi<R, K, PREC>), grid, dim3(kNT), bytes, s, P, HY, WMAX, NNMAX);
  return hipGetLastError();
}

template <typename R, bool PREC>
static hipError_t launch_tdi_k(const TdiLaunch& P, hipStream_t s) {
  switch (P.taps) {
    case 2: return launch_tdi_t<R, 2, PREC>(P, s);
    case 4: return launch_tdi_t<R, 4, PREC>(P, s);
    case 6: return launch_tdi_t<R, 6, PREC>(P, s);
    case 8: return launch_tdi_t<R, 8, PREC>(P, s);
    case 12: return launch_tdi_t<R, 12, PREC>(P, s);
    case 16: return launch_tdi_t<R, 16, PREC>(P, s);
    case 24: return launch_tdi_t<R, 24, PREC>(P, s);
    case 32: return launch_tdi_t<R, 32, PREC>(P, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_tdi(const TdiLaunch& P, hipStream_t s) {
  if (P.precision == 0)
    return P.precessing ? launch_tdi_k<double, true>(P, s) : launch_tdi_k<double, false>(P, s);
  return P.precessing ? launch_tdi_k<float, true>(P, s) : launch_tdi_k<float, false>(P, s);
}

}  // namespace lt
