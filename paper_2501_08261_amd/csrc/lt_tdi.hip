// Per-template setup, mode / polarisation kernels, and the fused TDI response
// kernel (hot-path steps a1-a8 of the time-domain LISA likelihood).
#include <algorithm>

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

// The same on a grid of twice the step: a workgroup evaluates the waveform at kNT even
// samples 2m (m = m0 .. m0 + kNT - 1, LDS) and writes the fine samples 2m and 2m + 1 for
// the first kNT - 1 of them, the odd one as the mean of its two neighbours.
template <typename R, bool PREC>
__global__ __launch_bounds__(kNT) void k_wave_coarse(const TplConst* tc, int mode_mask, GridDev g, R* h) {
  __shared__ cx<R> hv[kNT];
  const int b = blockIdx.y;
  const int64_t m = (int64_t)blockIdx.x * (kNT - 1) + threadIdx.x;
  const int64_t n = 2 * m;
  const TplConst& c = tc[b];
  cx<R> v{(R)0, (R)0};
  if (c.valid != 0.0 && (double)n >= c.n_start - 1.0 && n <= g.n)
    v = polarization_t<R, PREC>(c, mode_mask, g.t0 + (double)n * g.dt);
  hv[threadIdx.x] = v;
  __syncthreads();
  if (threadIdx.x == kNT - 1) return;
  const cx<R> w = hv[threadIdx.x + 1];
  if (n < g.n) {
    h[(2 * (int64_t)b) * g.n + n] = v.re;
    h[(2 * (int64_t)b + 1) * g.n + n] = -v.im;
  }
  if (n + 1 < g.n) {
    h[(2 * (int64_t)b) * g.n + n + 1] = (R)0.5 * (v.re + w.re);
    h[(2 * (int64_t)b + 1) * g.n + n + 1] = -((R)0.5 * (v.im + w.im));
  }
}

template <typename R>
static hipError_t launch_wave_t(const TplConst* tc, int64_t batch, int mode_mask, int precessing, int coarse,
                                GridDev g, R* h, hipStream_t s) {
  if (coarse == 2) {
    dim3 grid((unsigned)((g.n + 2 * (kNT - 1) - 1) / (2 * (kNT - 1))), (unsigned)batch);
    if (precessing)
      hipLaunchKernelGGL((k_wave_coarse<R, true>), grid, dim3(kNT), 0, s, tc, mode_mask, g, h);
    else
      hipLaunchKernelGGL((k_wave_coarse<R, false>), grid, dim3(kNT), 0, s, tc, mode_mask, g, h);
    return hipGetLastError();
  }
  dim3 grid((unsigned)((g.n + kNT - 1) / kNT), (unsigned)batch);
  if (precessing)
    hipLaunchKernelGGL((k_wave<R, true>), grid, dim3(kNT), 0, s, tc, mode_mask, g, h);
  else
    hipLaunchKernelGGL((k_wave<R, false>), grid, dim3(kNT), 0, s, tc, mode_mask, g, h);
  return hipGetLastError();
}

hipError_t launch_polarizations(const TplConst* tc, int64_t batch, int mode_mask, int precessing, int coarse,
                                GridDev g, double* hpc, hipStream_t s) {
  return launch_wave_t<double>(tc, batch, mode_mask, precessing, coarse, g, hpc, s);
}

hipError_t launch_wave(const TplConst* tc, int64_t batch, int mode_mask, int precessing, int coarse, int precision,
                       GridDev g, void* h, hipStream_t s) {
  if (precision == 0) return launch_wave_t<double>(tc, batch, mode_mask, precessing, coarse, g, (double*)h, s);
  return launch_wave_t<float>(tc, batch, mode_mask, precessing, coarse, g, (float*)h, s);
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

// One series at fractional index s.  FP64: the product form
//   sum_i c_i y_i prod_{j != i} d_j,  d_j = f - o_j,  c_i = 1 / prod_{j != i}(o_i - o_j),
// accumulated left to right: S_i = S_{i-1} d_i + c_i y_i P_{i-1}, P_i = P_{i-1} d_i.
// FP32: explicit weights first.  Its partial sums start at c_0 y_0, and with
// c_0 = 1/(K-1)! ~ 1e-34 at K = 32 and strain-sized y ~ 1e-21 that product
// is below the FP32 range; the weights themselves are O(1).
// ysh > 0: element i of the series sits at a[i + (i >> ysh)] (the padded link series of the
// FP64 response kernel)
template <int YSH>
__device__ inline int ypos(int i) {
  return YSH ? i + (i >> YSH) : i;
}

template <typename R, int K, int YSH = 0>
__device__ inline R lag1(const R* a, int len, double s) {
  double fl = floor(s);
  const R f = (R)(s - fl);
  const int j0 = stencil_start<K>(fl, len);
  if constexpr (YSH > 0) {
    // FP64 product form (see below) over the padded series
    constexpr LagDen<K> den;
    R P = f - (R)(-K / 2 + 1);
    R S = (R)den.inv[0] * a[ypos<YSH>(j0)];
#pragma unroll
    for (int i = 1; i < K; ++i) {
      const R d = f - (R)(i - K / 2 + 1);
      S = S * d + (R)den.inv[i] * a[ypos<YSH>(j0 + i)] * P;
      P *= d;
    }
    return S;
  }
  const R* p = a + j0;
  if (sizeof(R) == 4) {
    R w[K];
    lag_weights<R, K>(f, w);
    R acc = (R)0;
#pragma unroll
    for (int i = 0; i < K; ++i) acc += w[i] * p[i];
    return acc;
  }
  constexpr LagDen<K> den;
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

// Per node: for each link (N+, Nx, D_s, 1 - k.n), then D_r for each spacecraft; a node record
// adds the window bounds of its nine delays, ceil(D_max / dt) and floor(D_min / dt), as two
// int32, and the smallest 1 - k.n of its links.
constexpr int kNL = 4;
constexpr int kNodeVals = 6 * kNL + 3;
constexpr int kNodeRec = kNodeVals + 2;
// Below this 1 - k.n, somewhere among a tile's nodes, the response kernel interpolates N+, Nx
// and 1 - k.n separately and divides per sample; above it (every sky position more than ~11
// degrees from the arms over the tile) the quotients P = N / (1 - k.n) are smooth enough to be
// interpolated themselves.
constexpr double kSmoothKn = 0.02;
// receiver spacecraft (0-based) of links 1, 2, 3, -1, -2, -3; a compile-time function, so that in
// the unrolled link loops the receiver's interpolated h is picked by register, not by a select
__host__ __device__ constexpr int recv_sc(int li) {
  return li == 0 ? 1 : li == 1 ? 2 : li == 2 ? 0 : li == 3 ? 2 : li == 4 ? 0 : 1;
}
__constant__ int kRecvLink[3] = {2, 0, 1};          // a link received by spacecraft 1, 2, 3

// ------------------------------------------------------- response geometry per (template, orbit node)
// Projection numerators N+ = ((u.n)^2 - (v.n)^2) / 2, Nx = (u.n)(v.n), the denominator 1 - k.n
// and the delays D_s = L + k.r_s / c (sender) and D_r = k.r_r / c (receiver) of Eq. (2.8), at
// every node of the orbit table, computed once per template; [batch][n_nodes][kNodeRec] doubles.
// The three geometric factors are smooth in time and can be interpolated separately between
// the nodes; their quotient is not, where the wave travels almost along an arm (k.n -> 1: the
// quotient then turns through its range within a node interval, while y itself vanishes).
__device__ inline void node_record(const TplConst& c, const OrbitDev& orb, int j, double inv_dt, double* o) {
  int dhi = -(1 << 30), dlo = 1 << 30;
  double dmin = 2.0;
  for (int q = 0; q < 6; ++q) {
    const double* e = orb.tab + (int64_t)j * kNodeStride + q * kNodeLink;
    const double un = c.u[0] * e[7] + c.u[1] * e[8] + c.u[2] * e[9];
    const double vn = c.v[0] * e[7] + c.v[1] * e[8] + c.v[2] * e[9];
    const double kn = c.k[0] * e[7] + c.k[1] * e[8] + c.k[2] * e[9];
    const double dly = e[0] + (c.k[0] * e[4] + c.k[1] * e[5] + c.k[2] * e[6]);
    o[q * kNL + 0] = 0.5 * (un * un - vn * vn);
    o[q * kNL + 1] = un * vn;
    o[q * kNL + 2] = dly;
    o[q * kNL + 3] = 1.0 - kn;
    dmin = fmin(dmin, 1.0 - kn);
    dhi = max(dhi, (int)ceil(dly * inv_dt));
    dlo = min(dlo, (int)floor(dly * inv_dt));
  }
  for (int q = 0; q < 3; ++q) {
    const double* e = orb.tab + (int64_t)j * kNodeStride + kRecvLink[q] * kNodeLink;
    const double dly = c.k[0] * e[1] + c.k[1] * e[2] + c.k[2] * e[3];
    o[6 * kNL + q] = dly;
    dhi = max(dhi, (int)ceil(dly * inv_dt));
    dlo = min(dlo, (int)floor(dly * inv_dt));
  }
  int2 wb;
  wb.x = dhi;
  wb.y = dlo;
  *reinterpret_cast<int2*>(o + kNodeVals) = wb;
  o[kNodeVals + 1] = dmin;
}

// One record per (template, node).  The workgroup builds its kNT records in LDS and writes them
// as one contiguous block: stored by each thread directly, a store instruction touched 64
// records kNodeRec * 8 bytes apart, and the partial lines cost 2.7 times the record bytes in
// HBM writes.
__global__ __launch_bounds__(kNT) void k_nodes(const TplConst* tc, OrbitDev orb, double inv_dt, double* nodes) {
  __shared__ double rec[kNT * kNodeRec];
  const int j0 = blockIdx.x * kNT;
  const int j = j0 + threadIdx.x;
  const int b = blockIdx.y;
  if (j < orb.n_nodes) node_record(tc[b], orb, j, inv_dt, rec + threadIdx.x * kNodeRec);
  __syncthreads();
  const int nj = orb.n_nodes - j0 < kNT ? orb.n_nodes - j0 : kNT;
  double* dst = nodes + ((int64_t)b * orb.n_nodes + j0) * kNodeRec;
  for (int i = threadIdx.x; i < nj * kNodeRec; i += kNT) dst[i] = rec[i];
}

// window bounds of every (template, tile): the largest and smallest delay in samples over
// the orbit nodes the tile interpolates (nodes jn_lo .. jn_hi, as in k_tdi), and whether the
// projection quotients are smooth over them (1 - k.n >= kSmoothKn on every link), four int32
__global__ __launch_bounds__(kNT) void k_windows(const double* nodes, OrbitDev orb, int64_t batch, int ntile,
                                                 int HY, int MY, int* win, unsigned long long* counter) {
  const int64_t idx = (int64_t)blockIdx.x * kNT + threadIdx.x;
  if (idx == 0) *counter = 0ull;   // the persistent response kernel's item counter
  if (idx >= batch * ntile) return;
  const int64_t b = idx / ntile, tile = idx - b * ntile;
  constexpr int S = kTile / (kTile / 256);
  const int64_t m_lo = tile * kTile - HY, m_hi = m_lo + MY - 1;
  const int64_t jn_lo = floordiv(m_lo, S) - 1 + orb.j0, jn_hi = floordiv(m_hi, S) + 2 + orb.j0;
  int dhi = -(1 << 30), dlo = 1 << 30;
  double dmin = 2.0;
  for (int64_t j = jn_lo; j <= jn_hi; ++j) {
    const double* rec = nodes + (b * orb.n_nodes + j) * kNodeRec;
    const int2 wb = *reinterpret_cast<const int2*>(rec + kNodeVals);
    dhi = max(dhi, wb.x);
    dlo = min(dlo, wb.y);
    dmin = fmin(dmin, rec[kNodeVals + 1]);
  }
  win[4 * idx] = dhi;
  win[4 * idx + 1] = dlo;
  win[4 * idx + 2] = dmin >= kSmoothKn ? 1 : 0;
  win[4 * idx + 3] = 0;
}

// ------------------------------------------------------- TDI term references per tile
// Per (TDI term, node interval) reference: the stencil start and fraction at
// the interval midpoint; the fraction of output n is f0 - delta(n) with
// delta(n) = (D(t_n) - D(t_ref)) / dt, cubic in the node values dn (FP64
// path) or linear, beta (n - n_ref), in mixed precision: the delays are sums
// of light times, whose second derivative moves delta by < 1e-9 samples over
// half an interval.
// Mixed precision, combined filters: the terms of one channel that read the
// same link are merged per interval into two filters over that link,
//   F = sum_t s_t c0_t (shifted to the term's stencil),
//   G = sum_t s_t beta_t c1_t,
// so that sum_t s_t y(n - D_t(n)) = (F * y)(n) - (n - n_ref) (G * y)(n),
// with c0, c1 the first-order Taylor weights of each term.
// The TDI delays are sums of arm light times, so all of this depends on the tile
// and the orbit only: it is built once per launch, one workgroup per tile, and every
// template's workgroup of that tile reads it.
constexpr int kTerms = 48;          // 3 channels x at most 16 terms
constexpr int kGroups = 12;         // 3 channels x at most 4 links
constexpr int kNV = kTile / 256;    // node intervals per tile (node spacing 256)
constexpr int kYPad = 8;            // zero samples after each y series
template <int K>
struct CombLen {
  static constexpr int value = ((K + 16 + 3) / 4) * 4;   // filter length bound (multiple of 4)
};

// byte layout of one tile's record
template <typename R, int K>
struct RefLayout {
  static constexpr int JMAX = CombLen<K>::value;
  static constexpr bool TAY = sizeof(R) == 4 && K <= 16;       // first-order weights (mixed, K <= 16)
  static constexpr size_t f0 = 0;                                             // double [kTerms * kNV]
  static constexpr size_t jr = f0 + sizeof(double) * kTerms * kNV;             // int [kTerms * kNV]
  static constexpr size_t tdn = jr + sizeof(int) * kTerms * kNV;               // R [kTerms * kNV * (TAY ? 1 : 4)]
  static constexpr size_t flag = tdn + sizeof(R) * kTerms * kNV * (TAY ? 1 : 4);   // uchar [kTerms * kNV]
  static constexpr size_t gj = (flag + kTerms * kNV + 15) & ~(size_t)15;       // int [kGroups * kNV] start, length
  static constexpr size_t comb = gj + sizeof(int) * 2 * kGroups * kNV;         // int: combined filters usable
  static constexpr size_t fg = (comb + sizeof(int) + 15) & ~(size_t)15;        // R G [kGroups * kNV][JMAX]
  static constexpr size_t fd = (fg + (TAY ? sizeof(R) * kGroups * kNV * JMAX : 0) + 31) & ~(size_t)31;
  //                                                                          double F [kGroups * kNV][JMAX]
  static constexpr size_t stride = (fd + (TAY ? sizeof(double) * kGroups * kNV * JMAX : 0) + 255) & ~(size_t)255;
};

template <typename R, int K, bool TAY>
__global__ __launch_bounds__(kNT) void k_tdi_refs(TdiLaunch P, int HY, int MYP, int comb) {
  using Lay = RefLayout<R, K>;
  constexpr int JMAX = Lay::JMAX;
  __shared__ double tf0[kTerms * kNV];
  __shared__ int tjr[kTerms * kNV];
  __shared__ R tdn[kTerms * kNV * (TAY ? 1 : 4)];
  __shared__ unsigned char tflag[kTerms * kNV];
  __shared__ int gj0[kGroups * kNV], gJ[kGroups * kNV];
  __shared__ __align__(16) R fg[TAY ? kGroups * kNV * 2 * JMAX : 4];
  __shared__ double fgd[TAY ? kGroups * kNV * JMAX : 1];     // F summed in FP64
  __shared__ int s_comb, s_span_bad;
  const int tid = threadIdx.x;
  const int64_t n0 = (int64_t)blockIdx.x * kTile;
  const int64_t m_lo = n0 - HY;
  constexpr int S = kTile / kNV;
  const double inv_dt = P.g.inv_dt;
  for (int i = tid; i < kGroups * kNV; i += kNT) gj0[i] = gJ[i] = 0;
  if (tid == 0) {
    s_comb = comb;
    s_span_bad = 0;
  }
  __syncthreads();
  // E: per (term, interval) references for the TDI delays
  const int S2 = S / 2;
  for (int e = tid; e < kTerms * kNV; e += kNT) {
    const int tg = e / kNV, v = e - tg * kNV;
    const int cc = tg >> 4, t = tg & 15;
    if (t >= P.terms.n_terms[cc]) continue;
    const Term& tm = P.terms.t[cc][t];
    const int64_t nv0 = n0 + (int64_t)v * S;
    const int64_t jg = floordiv(nv0, S) + P.orb.j0;   // orbit node at the interval start
    double D[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double a = 0.0;
      for (int k = 0; k < tm.nd; ++k)
        a += (double)tm.dcnt[k] * P.orb.tab[(jg - 1 + r) * kNodeStride + tm.dlink[k] * kNodeLink];
      D[r] = a;
    }
    // cubic interpolant at the interval midpoint (weights -1/16, 9/16, 9/16, -1/16)
    const double Dref = (-D[0] + 9.0 * D[1] + 9.0 * D[2] - D[3]) * 0.0625;
    const double sref = (double)(nv0 + S2 - m_lo) - Dref * inv_dt;
    const double fl = floor(sref);
    const double f0 = sref - fl;
    double db = 0.0, dnr[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      dnr[r] = (D[r] - Dref) * inv_dt;
      if (!TAY) tdn[e * 4 + r] = (R)dnr[r];
      db = fmax(db, fabs(dnr[r]));
    }
    // delay rate at the midpoint (derivative of the cubic node interpolant), samples per sample
    if (TAY) tdn[e] = (R)(((dnr[0] - dnr[3]) * (1.0 / 24.0) + (dnr[2] - dnr[1]) * 1.125) / (double)S);
    db *= 1.25;   // bound of the cubic interpolant over the interval
    // first-order weights are exact to 1.6 K delta^2 relative: keep that below 2e-8
    const double thr = TAY ? sqrt(2e-8 / (1.6 * K)) : -1.0;
    int flag;
    if (tm.nd == 0) flag = 2;
    else if (db <= thr && f0 - db >= 0.0 && f0 + db < 1.0) flag = 0;
    else flag = 1;
    if (flag == 1) s_comb = 0;
    tf0[e] = f0;
    tjr[e] = (int)fl;
    tflag[e] = flag;
  }
  __syncthreads();
  // F: combined filters per (channel, link group, interval) -- mixed precision only
  int comb1 = 0;
  if (TAY) {
    const int comb0 = s_comb;     // final after the barrier above
    if (comb0) {
      for (int gi = tid; gi < kGroups * kNV; gi += kNT) {
        const int cg = gi / kNV, v = gi - cg * kNV, cc = cg >> 2, g = cg & 3;
        int lo = 0, hi = 0;
        if (g < P.terms.n_groups[cc]) {
          const int nrefl = v * S + S2 + HY;          // n_ref - m_lo
          lo = 1 << 30;
          hi = -(1 << 30);
          for (int q = 0; q < P.terms.g_n[cc][g]; ++q) {
            const int e = (cc * 16 + P.terms.g_t[cc][g][q]) * kNV + v;
            const int bq = tflag[e] == 2 ? nrefl : tjr[e] - K / 2 + 1;
            lo = min(lo, bq);
            hi = max(hi, bq + (tflag[e] == 2 ? 1 : K));
          }
          lo &= ~3;     // 16-byte aligned start (lo > 128 > 0): the leading taps are zero
          // every read of phase D stays in [0, MYP): outputs sit within [-128, 124] of n_ref and
          // the last 4-tap block reads 8 samples
          if (hi - lo > JMAX || lo - 128 < 0 || hi + 132 > MYP) s_span_bad = 1;
        }
        gj0[gi] = lo;
        gJ[gi] = hi - lo;
      }
    }
    __syncthreads();
    comb1 = comb0 && !s_span_bad;
    if (comb1) {
      // each term adds its first-order weights c0, c1 (products of (f0 + x - o_j), j != i,
      // truncated after x) to its group's filters, one term of every group per round: the sums
      // run in term order
      for (int i = tid; i < kGroups * kNV * 2 * JMAX; i += kNT) fg[i] = (R)0;
      for (int i = tid; i < kGroups * kNV * JMAX; i += kNT) fgd[i] = 0.0;
      int qmax = 0;
      for (int cc = 0; cc < 3; ++cc)
        for (int g = 0; g < P.terms.n_groups[cc]; ++g) qmax = max(qmax, P.terms.g_n[cc][g]);
      __syncthreads();
      constexpr LagDen<K> den;
      for (int q = 0; q < qmax; ++q) {
        for (int item = tid; item < kGroups * kNV * K; item += kNT) {
          const int gi = item / K, i = item - gi * K;
          const int cg = gi / kNV, v = gi - cg * kNV, cc = cg >> 2, g = cg & 3;
          if (g >= P.terms.n_groups[cc] || q >= P.terms.g_n[cc][g]) continue;
          const int t = P.terms.g_t[cc][g][q];
          const int e = (cc * 16 + t) * kNV + v;
          const R sg = (R)P.terms.t[cc][t].sign;
          const double sgd = (double)P.terms.t[cc][t].sign;
          R* F = fg + (gi * 2) * JMAX;
          double* Fd = fgd + gi * JMAX;
          if (tflag[e] == 2) {
            if (i == 0) Fd[v * S + S2 + HY - gj0[gi]] += sgd;   // n_ref - m_lo, relative to the start
            continue;
          }
          const double f0 = tf0[e];
          double c0 = den.inv[i], c1 = 0.0;
          for (int j = 0; j < K; ++j) {
            if (j == i) continue;
            const double aj = f0 - (double)(j - K / 2 + 1);
            c1 = c1 * aj + c0;
            c0 = c0 * aj;
          }
          const int at = tjr[e] - K / 2 + 1 + i - gj0[gi];
          Fd[at] += sgd * c0;
          F[JMAX + at] += sg * tdn[e] * (R)c1;
        }
        __syncthreads();
      }
    }
    __syncthreads();
  }

  // the record
  unsigned char* rec = (unsigned char*)P.refs + (size_t)blockIdx.x * Lay::stride;
  for (int i = tid; i < kTerms * kNV; i += kNT) {
    ((double*)(rec + Lay::f0))[i] = tf0[i];
    ((int*)(rec + Lay::jr))[i] = tjr[i];
    (rec + Lay::flag)[i] = tflag[i];
  }
  for (int i = tid; i < kTerms * kNV * (TAY ? 1 : 4); i += kNT) ((R*)(rec + Lay::tdn))[i] = tdn[i];
  for (int i = tid; i < kGroups * kNV; i += kNT) {
    ((int*)(rec + Lay::gj))[i] = gj0[i];
    ((int*)(rec + Lay::gj))[kGroups * kNV + i] = gJ[i];
  }
  if (tid == 0) *(int*)(rec + Lay::comb) = comb1;
  if (TAY && comb1)
    // F stays FP64: the TDI 2.0 filters cancel the signal to (2 pi f L)^2 of y and below at
    // low frequencies, and an FP32 rounding of every tap (an error the same for all outputs of
    // the interval) would not cancel with it.  G only carries the delay drift (~1e-5 of F's
    // contribution) and is FP32.
    for (int i = tid; i < kGroups * kNV * JMAX; i += kNT) {
      const int gi = i / JMAX, j = i - gi * JMAX;
      ((double*)(rec + Lay::fd))[i] = fgd[i];
      ((R*)(rec + Lay::fg))[i] = fg[(gi * 2 + 1) * JMAX + j];
    }
}

// ------------------------------------------------------- fused TDI kernel
// One workgroup = one template x one tile of kTile output samples.
//  B: the template's node records covering the tile (LDS, FP64)
//  A: h+, hx on the window of grid samples the six links read (LDS)
//  C: y_slr for the tile plus the TDI halos; h is interpolated with K taps at
//     the three receiver and the six sender times (LDS)
//  D: X, Y, Z from y at the TDI delays (the tile's combined filters, read as scalars from
//     its record, or per term), then A, E, T (global)
template <typename R, int K, bool TAY>
__device__ __forceinline__ void tdi_item(const TdiLaunch& P, int HY, int WMAX, int NNMAX, int64_t ntile,
                                         int64_t tile, int b, unsigned char* smem) {
  using Lay = RefLayout<R, K>;
  constexpr int JMAX = Lay::JMAX;
  const int tid = threadIdx.x;
  const int64_t N = P.g.n;
  const int64_t n0 = tile * kTile;
  const TplConst& c = P.tc[b];
  // the likelihood discards a faulted template's residual: nothing to write
  if (P.out_mode == 2 && c.valid == 0.0) return;
  // y is needed on [n0 - HY, n0 + kTile + K/2]: the centred stencils of the
  // shortest TDI delays reach K/2 - 1 samples past the last output sample
  const int MY = kTile + HY + K / 2 + 1;
  const int MYP = (MY + kYPad + 3) & ~3;   // multiple of 4: aligned vector reads in phase D
  // FP64: a spare slot after every 16 samples of a link series.  Phase D's per-term reads have
  // lanes four samples (32 bytes) apart, which without the slots put four lanes of a 16-lane
  // group on each bank pair; with them the 16 lanes meet 16 different pairs
  constexpr int YSH = sizeof(R) == 8 ? 4 : 0;
  const int MYR = MYP + (YSH ? MYP >> YSH : 0);   // row stride of the link series in LDS
  R* yb = (R*)smem;
  R* hpb = yb + 6 * MYR;
  R* hxb = hpb + WMAX;
  double* nd = (double*)(smem + (((size_t)(6 * MYR + 2 * WMAX) * sizeof(R) + 15) & ~(size_t)15));
  // FP32 copies of the node geometry (mixed precision: it scales an FP32 product): P+, Px per
  // link (12 per node) where the tile is smooth, else N+, Nx, 1 - k.n (18 per node)
  float* ndp = (float*)(nd + NNMAX * kNodeVals);
  const unsigned char* rec = (const unsigned char*)P.refs + (size_t)tile * Lay::stride;
  const double* tf0 = (const double*)(rec + Lay::f0);
  const int* tjr = (const int*)(rec + Lay::jr);
  const R* tdn = (const R*)(rec + Lay::tdn);
  const unsigned char* tflag = rec + Lay::flag;
  const double inv_dt = P.g.inv_dt;
  const int64_t m_lo = n0 - HY, m_hi = m_lo + MY - 1;
  constexpr int S = kTile / kNV;   // node spacing (the launch checks that the table uses it)
  const int S2 = S / 2;
  const int64_t jn_lo = floordiv(m_lo, S) - 1 + P.orb.j0;
  const int64_t jn_hi = floordiv(m_hi, S) + 2 + P.orb.j0;
  const int NN = (int)(jn_hi - jn_lo + 1);

  // the tile's window bounds (k_windows): largest and smallest delay over its nodes, in samples
  typedef const __attribute__((address_space(4))) int cwin_t;
  cwin_t* wp = (cwin_t*)(P.win + 4 * ((int64_t)b * ntile + tile));
  const int smooth = wp[2];
  const long long w0 = (long long)m_lo - wp[0] - K / 2 - 2;
  const long long w1 = (long long)m_hi - wp[1] + K / 2 + 2;
  int W = (int)(w1 - w0 + 1);
  if (W > WMAX) {
    W = WMAX;
    if (tid == 0 && P.status) P.status[b] = 3;
  }
  // every needed h sample precedes the f_low start (or the template is invalid): all zero
  const int skip = (c.valid == 0.0 || (double)w1 < c.n_start - 2.0) ? 1 : 0;

  if (!skip) {
    // B: the template's node records and A: the polarisations of the window, every load
    // issued before the first LDS store (one memory latency per kA * kNT samples)
    const double* ng = P.nodes + ((int64_t)b * P.orb.n_nodes + jn_lo) * kNodeRec;
    const int nval = NN * kNodeVals;
    double nv = 0.0;
    if (tid < nval) nv = ng[(tid / kNodeVals) * kNodeRec + tid % kNodeVals];
    for (int i = tid + kNT; i < nval; i += kNT) nd[i] = ng[(i / kNodeVals) * kNodeRec + i % kNodeVals];
    if constexpr (sizeof(R) == 4) {
      if (smooth) {
        for (int i = tid; i < NN * 12; i += kNT) {
          const double* o = ng + (i / 12) * kNodeRec + (i % 12 / 2) * kNL;
          ndp[i] = (float)(o[i & 1] / o[3]);
        }
      } else {
        for (int i = tid; i < NN * 18; i += kNT) {
          const int f = i % 3;
          ndp[i] = (float)ng[(i / 18) * kNodeRec + (i % 18 / 3) * kNL + (f == 2 ? 3 : f)];
        }
      }
    }
    constexpr int kA = 6;
    const R* hg = (const R*)P.h + (2 * (int64_t)b) * N;
    for (int i0 = 0; i0 < W; i0 += kA * kNT) {
      R vp[kA], vx[kA];
#pragma unroll
      for (int r = 0; r < kA; ++r) {
        const long long j = w0 + i0 + r * kNT + tid;
        const bool in = i0 + r * kNT + tid < W && j >= 0 && j < N;
        vp[r] = in ? hg[j] : (R)0;
        vx[r] = in ? hg[N + j] : (R)0;
      }
#pragma unroll
      for (int r = 0; r < kA; ++r) {
        const int i = i0 + r * kNT + tid;
        if (i < W) {
          hpb[i] = vp[r];
          hxb[i] = vx[r];
        }
      }
    }
    if (tid < nval) nd[tid] = nv;
    __syncthreads();
    // C: link responses y_slr for m in [m_lo, m_hi].  A thread's samples are kNT = S apart,
    // one node interval: they share the cubic node weights, and the node index steps by one.
    static_assert(kNT == S, "phase C strides by one node interval");
    const int64_t q0 = floordiv(m_lo + tid, S);
    double w[4];
    cubic_w((double)(m_lo + tid - q0 * S) / (double)S, w);
    const float wp[4] = {(float)w[0], (float)w[1], (float)w[2], (float)w[3]};
    const int jl0 = (int)(q0 + P.orb.j0 - jn_lo);
    for (int mi = tid, it = 0; mi < MY; mi += kNT, ++it) {
      int64_t m = m_lo + mi;
      if (m < 0 || m >= N) {
#pragma unroll
        for (int li = 0; li < 6; ++li) yb[li * MYR + ypos<YSH>(mi)] = (R)0;
        continue;
      }
      const double* o0 = nd + (jl0 + it - 1) * kNodeVals;
      const double mloc = (double)(m - w0);
      R hpr[3], hxr[3];
#pragma unroll
      for (int sc = 0; sc < 3; ++sc) {
        double Dr = 0.0;
#pragma unroll
        for (int r = 0; r < 4; ++r) Dr += w[r] * o0[r * kNodeVals + 6 * kNL + sc];
        lag2<R, K>(hpb, hxb, W, mloc - Dr * inv_dt, hpr[sc], hxr[sc]);
      }
      if (sizeof(R) == 4 && smooth) {
#pragma unroll
        for (int li = 0; li < 6; ++li) {
          R v0 = (R)0, v1 = (R)0;
          double v2 = 0.0;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const float* op = ndp + (jl0 + it - 1 + r) * 12 + 2 * li;
            v0 += wp[r] * op[0];
            v1 += wp[r] * op[1];
            v2 += w[r] * o0[r * kNodeVals + li * kNL + 2];
          }
          R hps, hxs;
          lag2<R, K>(hpb, hxb, W, mloc - v2 * inv_dt, hps, hxs);
          const int rc = recv_sc(li);
          yb[li * MYR + ypos<YSH>(mi)] = v0 * (hps - hpr[rc]) + v1 * (hxs - hxr[rc]);
        }
      } else {
#pragma unroll
        for (int li = 0; li < 6; ++li) {
          R v0 = (R)0, v1 = (R)0, v3 = (R)0;
          double v2 = 0.0;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const double* o = o0 + r * kNodeVals + li * kNL;
            if constexpr (sizeof(R) == 4) {
              const float* op = ndp + (jl0 + it - 1 + r) * 18 + 3 * li;
              v0 += wp[r] * op[0];
              v1 += wp[r] * op[1];
              v3 += wp[r] * op[2];
            } else {
              v0 += w[r] * o[0];
              v1 += w[r] * o[1];
              v3 += w[r] * o[3];
            }
            v2 += w[r] * o[2];
          }
          R hps, hxs;
          lag2<R, K>(hpb, hxb, W, mloc - v2 * inv_dt, hps, hxs);
          const int rc = recv_sc(li);
          const R num = v0 * (hps - hpr[rc]) + v1 * (hxs - hxr[rc]);
          if constexpr (sizeof(R) == 4)
            yb[li * MYR + ypos<YSH>(mi)] = num * __builtin_amdgcn_rcpf(v3);
          else
            yb[li * MYR + ypos<YSH>(mi)] = num / v3;
        }
      }
    }
    // zero the tail of each y series up to its padded length: filter taps beyond the data read it
    for (int i = tid; i < 6 * (MYP - MY); i += kNT)
      yb[(i / (MYP - MY)) * MYR + ypos<YSH>(MY + (i % (MYP - MY)))] = (R)0;
    __syncthreads();
  }

  // the tile's combined filters are read from its record in the constant address space: they
  // are the same for every lane of a wave (one wave = one node interval), so they arrive in
  // scalar registers and feed the multiply-adds as scalar operands
  typedef const __attribute__((address_space(4))) unsigned char crec_t;
  crec_t* crec = (crec_t*)rec;
  const int comb1 = (TAY && !skip) ? *(const __attribute__((address_space(4))) int*)(crec + Lay::comb) : 0;

  // D: TDI and A, E, T; each thread owns four consecutive output samples.  The channels
  // accumulate in FP64 in both precisions: the terms of a channel cancel against each other at
  // low frequencies, and X, Y and Z against each other in T, so FP32 rounding of their sums
  // would set the error of T, the channel with the lowest noise.
  const R* data = (const R*)P.data;
  R* out = (R*)P.out;
  const int nl0 = 4 * tid;
  const int64_t nb = n0 + nl0;
  if (nb >= N) return;
  double ch[3][4];
  R dv[3][4];
#pragma unroll
  for (int cc = 0; cc < 3; ++cc)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      ch[cc][k] = 0.0;
      // the data of the residual, loaded before the filters run
      dv[cc][k] = (P.out_mode == 2 && nb + k < N) ? data[cc * N + nb + k] : (R)0;
    }
  if (!skip) {
    const int v = nl0 / S;
    const int64_t nref = n0 + (int64_t)v * S + S2;
    if (TAY && comb1) {
      const int dn0 = (int)(nb - nref);
      const int vw = __builtin_amdgcn_readfirstlane(v);
      typedef float v4c __attribute__((ext_vector_type(4)));
      typedef const __attribute__((address_space(4))) int cint_t;
      typedef const __attribute__((address_space(4))) v4c cf4_t;
      cint_t* gjs = (cint_t*)(crec + Lay::gj);
      for (int cc = 0; cc < 3; ++cc) {
        for (int g = 0; g < P.terms.n_groups[cc]; ++g) {
          const int gi = (cc * 4 + g) * kNV + vw;
          const int J = gjs[kGroups * kNV + gi];
          static_assert(!TAY || YSH == 0, "combined filters read unpadded series");
          const R* yl = yb + P.terms.g_link[cc][g] * MYR + gjs[gi] + dn0;
          typedef double v4d __attribute__((ext_vector_type(4)));
          typedef const __attribute__((address_space(4))) v4d cd4_t;
          cd4_t* F = (cd4_t*)(crec + Lay::fd + (size_t)gi * JMAX * sizeof(double));
          cf4_t* G = (cf4_t*)(crec + Lay::fg + (size_t)gi * JMAX * sizeof(R));
          // F's products and sums in FP64 (y is exact in FP64); the drift term in FP32
          double a[4] = {0.0, 0.0, 0.0, 0.0};
          R d[4] = {(R)0, (R)0, (R)0, (R)0};
          // yl, F, G and j are 16-byte aligned (gj0, MYP, JMAX and n - n_ref are multiples of 4):
          // one 16 B read of y per four taps, the window of eight samples kept in registers; eight
          // lanes of a 16 B read cover the 32 LDS banks without conflict
          // (volatile: the compiler would otherwise split the 16 B reads into 4 B reads that
          // conflict four ways)
          typedef float v4f __attribute__((ext_vector_type(4)));
          typedef const volatile __attribute__((address_space(3))) v4f lds_v4f;
          v4f y0 = *(lds_v4f*)(yl);
          double yd0[4] = {(double)y0.x, (double)y0.y, (double)y0.z, (double)y0.w};
          for (int j = 0; j < J; j += 4) {
            R yv[8];
            double yd[8];
            const v4f y1 = *(lds_v4f*)(yl + j + 4);
            yv[0] = y0.x; yv[1] = y0.y; yv[2] = y0.z; yv[3] = y0.w;
            yv[4] = y1.x; yv[5] = y1.y; yv[6] = y1.z; yv[7] = y1.w;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              yd[i] = yd0[i];
              yd[4 + i] = (double)yv[4 + i];
              yd0[i] = yd[4 + i];
            }
            y0 = y1;
            const v4d f4 = F[j / 4];
            const v4c g4 = G[j / 4];
            const double fa[4] = {f4.x, f4.y, f4.z, f4.w};
            const R ga[4] = {g4.x, g4.y, g4.z, g4.w};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
#pragma unroll
              for (int k = 0; k < 4; ++k) {
                a[k] = fma(fa[i], yd[i + k], a[k]);
                d[k] += ga[i] * yv[i + k];
              }
            }
          }
#pragma unroll
          for (int k = 0; k < 4; ++k) ch[cc][k] += a[k] - (double)((R)(dn0 + k) * d[k]);
        }
      }
    } else {
    R cw[4][4];
    if (!TAY) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        double w[4];
        cubic_w((double)(nl0 - v * S + k) / (double)S, w);
#pragma unroll
        for (int r = 0; r < 4; ++r) cw[k][r] = (R)w[r];
      }
    }
    for (int cc = 0; cc < 3; ++cc) {
      for (int t = 0; t < P.terms.n_terms[cc]; ++t) {
        const Term& tm = P.terms.t[cc][t];
        const int e = (cc * 16 + t) * kNV + v;
        const R* yl = yb + tm.link * MYR;
        const int flag = tflag[e];
        R val[4];
        if (flag == 2) {
#pragma unroll
          for (int k = 0; k < 4; ++k) val[k] = yl[ypos<YSH>((int)(nb + k - m_lo))];
        } else {
          R dl[4];
          if (TAY) {
#pragma unroll
            for (int k = 0; k < 4; ++k) dl[k] = tdn[e] * (R)(nb + k - nref);
          } else {
#pragma unroll
            for (int k = 0; k < 4; ++k)
              dl[k] = cw[k][0] * tdn[e * 4] + cw[k][1] * tdn[e * 4 + 1] + cw[k][2] * tdn[e * 4 + 2] +
                      cw[k][3] * tdn[e * 4 + 3];
          }
          const int jb = tjr[e] + (int)(nb - nref);
          const double f0 = tf0[e];
#pragma unroll
          for (int k = 0; k < 4; ++k) val[k] = lag1<R, K, YSH>(yl, MY, (double)(jb + k) + (f0 - (double)dl[k]));
        }
        if (tm.sign > 0) {
#pragma unroll
          for (int k = 0; k < 4; ++k) ch[cc][k] += val[k];
        } else {
#pragma unroll
          for (int k = 0; k < 4; ++k) ch[cc][k] -= val[k];
        }
      }
    }
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t n = nb + k;
    if (n >= N) break;
    R o0, o1, o2;
    if (P.out_mode == 1) {
      o0 = (R)ch[0][k]; o1 = (R)ch[1][k]; o2 = (R)ch[2][k];
    } else {
      // no contraction: A, E, T are formed in FP64 and rounded to R before the data is
      // subtracted, so a template equal to the data leaves a residual of exactly zero
#pragma clang fp contract(off)
      const double r2 = 0.70710678118654752440, r6 = 0.40824829046386301637, r3 = 0.57735026918962576451;
      o0 = (R)((ch[2][k] - ch[0][k]) * r2);
      o1 = (R)((ch[0][k] - 2.0 * ch[1][k] + ch[2][k]) * r6);
      o2 = (R)((ch[0][k] + ch[1][k] + ch[2][k]) * r3);
      o0 -= dv[0][k];   // zero unless the residual is written
      o1 -= dv[1][k];
      o2 -= dv[2][k];
    }
    const int64_t base = (int64_t)b * 3 * N + n;
    out[base] = o0;
    out[base + N] = o1;
    out[base + 2 * N] = o2;
  }
}

// Work item i of a launch (tile-major): template (i mod batch + tile) mod batch of tile
// i / batch when `rotate`, else template i mod batch.  Consecutive items share a tile, so that
// its record stays in L2; with the rotation, the round-robin placement of workgroups on the
// XCDs gives each XCD every template (lengths differ) over the tiles.
__device__ inline void tdi_item_index(const TdiLaunch& P, int64_t i, int64_t* tile, int* b) {
  *tile = i / P.batch;
  const int64_t r = i - *tile * P.batch;
  *b = (int)(P.rotate ? (r + *tile) % P.batch : r);
}

// one workgroup per item
template <typename R, int K, bool TAY>
__global__ __launch_bounds__(kNT) void k_tdi(TdiLaunch P, int HY, int WMAX, int NNMAX) {
  extern __shared__ __align__(16) unsigned char smem[];
  int64_t tile;
  int b;
  tdi_item_index(P, (int64_t)blockIdx.y * gridDim.x + blockIdx.x, &tile, &b);
  tdi_item<R, K, TAY>(P, HY, WMAX, NNMAX, gridDim.x, tile, b, smem);
}

// persistent: a fixed grid whose workgroups take items from a counter until none is left (the
// counter is zeroed by k_windows, which runs before on the same stream).  Every thread of a
// workgroup runs the same items and meets the same barriers; the loop ends for all of them
// when the counter passes the last item.
template <typename R, int K, bool TAY>
__global__ __launch_bounds__(kNT) void k_tdi_persistent(TdiLaunch P, int HY, int WMAX, int NNMAX, int ntile) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int64_t s_item;
  const int64_t total = (int64_t)ntile * P.batch;
  for (;;) {
    __syncthreads();                   // the previous item is done with the LDS and s_item
    if (threadIdx.x == 0) s_item = (int64_t)atomicAdd((unsigned long long*)P.counter, 1ull);
    __syncthreads();
    const int64_t i = s_item;
    if (i >= total) break;
    int64_t tile;
    int b;
    tdi_item_index(P, i, &tile, &b);
    tdi_item<R, K, TAY>(P, HY, WMAX, NNMAX, ntile, tile, b, smem);
  }
}

// launch geometry of the response kernel (host)
template <typename R, int K>
struct TdiGeom {
  int HY, MYP, WMAX, NNMAX, comb;
  unsigned ntile;
  size_t bytes;
  hipError_t make(const TdiLaunch& P) {
    constexpr bool TAY = RefLayout<R, K>::TAY;
    HY = (int)ceil(7.0 * P.orb.max_light_time * P.g.inv_dt * 1.001) + K / 2 + 2;
    const int spread = (int)ceil(2.0 * P.orb.max_light_time * P.g.inv_dt * 1.01) + 8;
    const int MY = kTile + HY + K / 2 + 1;
    MYP = (MY + kYPad + 3) & ~3;
    WMAX = MY + spread + K + 8;
    NNMAX = MY / P.orb.spacing + 5;
    if (HY + 8 > P.orb.spacing || K / 2 + 9 > P.orb.spacing) return hipErrorInvalidValue;   // node table covers one spacing of halo
    if (P.orb.spacing * kNV != kTile) return hipErrorInvalidValue;
    if (!P.nodes || !P.refs) return hipErrorInvalidValue;
    constexpr int JMAX = CombLen<K>::value;
    const int MYR = MYP + (sizeof(R) == 8 ? MYP / 16 : 0);   // padded link series (FP64)
    bytes = (((size_t)(6 * MYR + 2 * WMAX) * sizeof(R) + 15) & ~(size_t)15) + (size_t)NNMAX * kNodeVals * sizeof(double) +
            (sizeof(R) == 4 ? (size_t)NNMAX * 18 * sizeof(float) : 0);
    if (bytes > 160 * 1024) return hipErrorInvalidValue;
    // combined filters: a group spans its delay range plus one stencil plus up to 3 alignment taps
    const int span = (int)ceil(P.terms.g_span * P.orb.max_light_time * P.g.inv_dt * 1.001) + 2 + K + 3;
    comb = (TAY && P.comb && span <= JMAX) ? 1 : 0;
    ntile = (unsigned)((P.g.n + kTile - 1) / kTile);
    return hipSuccess;
  }
};

template <typename R, int K>
static hipError_t launch_tdi_t(const TdiLaunch& P0, int stage, hipStream_t s) {
  constexpr bool TAY = RefLayout<R, K>::TAY;
  TdiLaunch P = P0;
  P.win = (int*)(P.nodes + (int64_t)P.batch * P.orb.n_nodes * kNodeRec);
  TdiGeom<R, K> G;
  hipError_t e = G.make(P);
  if (e != hipSuccess) return e;
  P.counter = (unsigned long long*)((unsigned char*)P.refs + (size_t)G.ntile * RefLayout<R, K>::stride);
  if (stage == 0) {
    hipLaunchKernelGGL(k_nodes, dim3((unsigned)((P.orb.n_nodes + kNT - 1) / kNT), (unsigned)P.batch), dim3(kNT), 0,
                       s, P.tc, P.orb, P.g.inv_dt, P.nodes);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nw = P.batch * (int64_t)G.ntile;
    hipLaunchKernelGGL(k_windows, dim3((unsigned)((nw + kNT - 1) / kNT)), dim3(kNT), 0, s, P.nodes, P.orb, P.batch,
                       (int)G.ntile, G.HY, kTile + G.HY + K / 2 + 1, P.win, P.counter);
    e = hipGetLastError();
    if (e != hipSuccess || P.refs_ready) return e;
    hipLaunchKernelGGL((k_tdi_refs<R, K, TAY>), dim3(G.ntile), dim3(kNT), 0, s, P, G.HY, G.MYP, G.comb);
    return hipGetLastError();
  }
  if (P.persistent) {
    e = hipFuncSetAttribute((const void*)k_tdi_persistent<R, K, TAY>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)G.bytes);
    if (e != hipSuccess) return e;
    int dev = 0, ncu = 0;
    e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const int64_t items = (int64_t)G.ntile * P.batch;
    int64_t wgs = (int64_t)ncu * (P.wg_per_cu > 0 ? P.wg_per_cu : 1);
    if (wgs > items) wgs = items;
    hipLaunchKernelGGL((k_tdi_persistent<R, K, TAY>), dim3((unsigned)wgs), dim3(kNT), G.bytes, s, P, G.HY, G.WMAX,
                       G.NNMAX, (int)G.ntile);
    return hipGetLastError();
  }
  e = hipFuncSetAttribute((const void*)k_tdi<R, K, TAY>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)G.bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_tdi<R, K, TAY>), dim3(G.ntile, (unsigned)P.batch), dim3(kNT), G.bytes, s, P, G.HY, G.WMAX,
                     G.NNMAX);
  return hipGetLastError();
}

template <typename R>
static size_t refs_stride_k(int taps) {
  switch (taps) {
    case 2: return RefLayout<R, 2>::stride;
    case 4: return RefLayout<R, 4>::stride;
    case 6: return RefLayout<R, 6>::stride;
    case 8: return RefLayout<R, 8>::stride;
    case 12: return RefLayout<R, 12>::stride;
    case 16: return RefLayout<R, 16>::stride;
    case 24: return RefLayout<R, 24>::stride;
    case 32: return RefLayout<R, 32>::stride;
    default: return 0;
  }
}

void tdi_scratch_bytes(const TdiLaunch& P, size_t* nodes, size_t* refs) {
  // node records, then two int32 window bounds per (template, tile)
  *nodes = (size_t)P.batch * (size_t)P.orb.n_nodes * kNodeRec * sizeof(double) +
           (size_t)P.batch * (size_t)((P.g.n + kTile - 1) / kTile) * 4 * sizeof(int);
  const size_t stride = P.precision == 0 ? refs_stride_k<double>(P.taps) : refs_stride_k<float>(P.taps);
  // the records, then the persistent kernel's item counter
  *refs = stride ? (size_t)((P.g.n + kTile - 1) / kTile) * stride + 256 : 0;
}

template <typename R>
static hipError_t launch_tdi_k(const TdiLaunch& P, int stage, hipStream_t s) {
  switch (P.taps) {
    case 2: return launch_tdi_t<R, 2>(P, stage, s);
    case 4: return launch_tdi_t<R, 4>(P, stage, s);
    case 6: return launch_tdi_t<R, 6>(P, stage, s);
    case 8: return launch_tdi_t<R, 8>(P, stage, s);
    case 12: return launch_tdi_t<R, 12>(P, stage, s);
    case 16: return launch_tdi_t<R, 16>(P, stage, s);
    case 24: return launch_tdi_t<R, 24>(P, stage, s);
    case 32: return launch_tdi_t<R, 32>(P, stage, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_tdi(const TdiLaunch& P, int stage, hipStream_t s) {
  return P.precision == 0 ? launch_tdi_k<double>(P, stage, s) : launch_tdi_k<float>(P, stage, s);
}

}  // namespace lt
