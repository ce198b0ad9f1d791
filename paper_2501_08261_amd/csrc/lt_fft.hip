// Batched real-to-complex FFT (hot-path step a9) and the band-limited inner
// products / log-likelihood (a10).
//
// A real series of length N is read as n = N/2 complex samples
// z_j = x_{2j} + i x_{2j+1}.  The length-n complex DFT is done in two passes
// (four-step, n = n1 * n2, j = n2 j1 + j2, k = k1 + n1 k2):
//   pass 1: for each column j2, a length-n1 DFT over j1, times exp(-2 pi i j2 k1 / n);
//   pass 2: for each row k1, a length-n2 DFT over j2 -> Z_{k1 + n1 k2}.
// Sub-DFTs run in LDS as mixed-radix (2, 3, 4, 5, 8) Stockham autosort stages.
// Pass 2 works on the row pair (k1, n1 - k1), which holds every mirror pair
// (k, n - k) needed to untangle the real transform:
//   X_k = (Z_k + conj Z_{n-k})/2 - (i/2) exp(-2 pi i k / N) (Z_k - conj Z_{n-k}),
// and either writes X_k * dt or accumulates sum_band |X_k|^2 / S_k in FP64.
#include "lt_kernels.hpp"

namespace lt {

constexpr int kFT = 256;

template <typename R> struct C2 { R x, y; };
template <typename R> __device__ inline C2<R> operator+(C2<R> a, C2<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R> __device__ inline C2<R> operator-(C2<R> a, C2<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R> __device__ inline C2<R> cm(C2<R> a, C2<R> b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
template <typename R> __device__ inline C2<R> mi(C2<R> a) { return {a.y, -a.x}; }   // -i a
template <typename R> __device__ inline C2<R> sc(C2<R> a, R s) { return {a.x * s, a.y * s}; }

template <typename R> __device__ inline const R* tw_ptr(const double* d, const float* f);
template <> __device__ inline const double* tw_ptr<double>(const double* d, const float*) { return d; }
template <> __device__ inline const float* tw_ptr<float>(const double*, const float* f) { return f; }

// forward DFT of size RAD in registers
template <typename R, int RAD> __device__ inline void dft(C2<R>* v);
template <typename R> __device__ inline void dft2(C2<R>* v) {
  C2<R> a = v[0], b = v[1];
  v[0] = a + b;
  v[1] = a - b;
}
template <typename R, int RAD> __device__ inline void dft(C2<R>* v) {
  if constexpr (RAD == 2) {
    dft2(v);
  } else if constexpr (RAD == 3) {
    const R s1 = (R)0.86602540378443864676;
    C2<R> t1 = v[1] + v[2], t2 = v[0] - sc(t1, (R)0.5), t3 = sc(mi(v[1] - v[2]), s1);
    v[0] = v[0] + t1;
    v[1] = t2 + t3;
    v[2] = t2 - t3;
  } else if constexpr (RAD == 4) {
    C2<R> a = v[0] + v[2], b = v[0] - v[2], c = v[1] + v[3], d = mi(v[1] - v[3]);
    v[0] = a + c;
    v[2] = a - c;
    v[1] = b + d;
    v[3] = b - d;
  } else if constexpr (RAD == 5) {
    const R c1 = (R)0.30901699437494742410, c2 = (R)-0.80901699437494742410;
    const R s1 = (R)0.95105651629515357212, s2 = (R)0.58778525229247312917;
    C2<R> a1 = v[1] + v[4], a2 = v[2] + v[3], b1 = v[1] - v[4], b2 = v[2] - v[3];
    C2<R> x0 = v[0];
    C2<R> p1 = x0 + sc(a1, c1) + sc(a2, c2), p2 = x0 + sc(a1, c2) + sc(a2, c1);
    C2<R> q1 = mi(sc(b1, s1) + sc(b2, s2)), q2 = mi(sc(b1, s2) - sc(b2, s1));
    v[0] = x0 + a1 + a2;
    v[1] = p1 + q1;
    v[4] = p1 - q1;
    v[2] = p2 + q2;
    v[3] = p2 - q2;
  } else if constexpr (RAD == 8) {
    C2<R> e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
    dft<R, 4>(e);
    dft<R, 4>(o);
    const R h = (R)0.70710678118654752440;
    C2<R> w1 = {h, -h}, w3 = {-h, -h};
    C2<R> t0 = o[0], t1 = cm(o[1], w1), t2 = mi(o[2]), t3 = cm(o[3], w3);
    v[0] = e[0] + t0; v[4] = e[0] - t0;
    v[1] = e[1] + t1; v[5] = e[1] - t1;
    v[2] = e[2] + t2; v[6] = e[2] - t2;
    v[3] = e[3] + t3; v[7] = e[3] - t3;
  } else if constexpr (RAD == 16) {
    // 16 = 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2.  A DFT-4 over n1 for each n2, the products
    // with exp(-2 pi i n2 k1 / 16), a DFT-4 over n2 for each k1
    const R c1 = (R)0.92387953251128675613, s1 = (R)0.38268343236508977173, h = (R)0.70710678118654752440;
    C2<R> y[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
#pragma unroll
      for (int n1 = 0; n1 < 4; ++n1) y[n2][n1] = v[4 * n1 + n2];
      dft<R, 4>(y[n2]);
    }
    y[1][1] = cm(y[1][1], C2<R>{c1, -s1});
    y[1][2] = cm(y[1][2], C2<R>{h, -h});
    y[1][3] = cm(y[1][3], C2<R>{s1, -c1});
    y[2][1] = cm(y[2][1], C2<R>{h, -h});
    y[2][2] = mi(y[2][2]);
    y[2][3] = cm(y[2][3], C2<R>{-h, -h});
    y[3][1] = cm(y[3][1], C2<R>{s1, -c1});
    y[3][2] = cm(y[3][2], C2<R>{-h, -h});
    y[3][3] = cm(y[3][3], C2<R>{-c1, s1});
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      C2<R> z[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
      dft<R, 4>(z);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = z[k2];
    }
  }
}

// Division of a non-negative value by a divisor that is the same for the whole workgroup: a
// shift when the divisor is a power of two (a uniform branch), else the integer division.
struct UDiv {
  int d, sh;
  __device__ explicit UDiv(int d_) : d(d_), sh((d_ & (d_ - 1)) == 0 ? __builtin_ctz((unsigned)d_) : -1) {}
  __device__ int div(int a) const { return sh >= 0 ? a >> sh : a / d; }
};

// One Stockham stage of radix RAD over `nfft` transforms of length L held in
// src (row-major [nfft][L]); writes dst.  tw: exp(-2 pi i k / L), k < L.
// P2: L is a power of two (then so are L / RAD and Ns): indices by shifts and masks.
template <typename R, int RAD, bool P2>
__device__ inline void stage(const C2<R>* src, C2<R>* dst, int L, int Ns, int nfft, const C2<R>* tw, int ls) {
  const int m = L / RAD;
  const int jobs = nfft * m;
  const int step = L / (Ns * RAD);
  const int lm = P2 ? __builtin_ctz((unsigned)m) : 0, lns = P2 ? __builtin_ctz((unsigned)Ns) : 0;
  for (int job = threadIdx.x; job < jobs; job += kFT) {
    int f, j, k, q;
    if constexpr (P2) {
      f = job >> lm;
      j = job & (m - 1);
      k = j & (Ns - 1);
      q = j >> lns;
    } else {
      f = job / m;
      j = job - f * m;
      q = j / Ns;
      k = j - q * Ns;
    }
    const C2<R>* s = src + f * ls;
    C2<R>* d = dst + f * ls;
    C2<R> v[RAD];
#pragma unroll
    for (int r = 0; r < RAD; ++r) {
      v[r] = s[j + r * m];
      if (r > 0 && k > 0) v[r] = cm(v[r], tw[r * k * step]);
    }
    dft<R, RAD>(v);
    int base = q * Ns * RAD + k;
#pragma unroll
    for (int r = 0; r < RAD; ++r) d[base + r * Ns] = v[r];
  }
}

// Full mixed-radix Stockham FFT in LDS over nfft transforms ls elements apart; returns the
// buffer holding the result.
template <typename R>
__device__ C2<R>* lds_fft(C2<R>* a, C2<R>* b, int L, const int* rad, int nr, int nfft, const C2<R>* tw, int ls) {
  int Ns = 1;
  const bool p2 = (L & (L - 1)) == 0;
  for (int s = 0; s < nr; ++s) {
    switch (rad[s]) {
      case 2:
        if (p2) stage<R, 2, true>(a, b, L, Ns, nfft, tw, ls);
        else stage<R, 2, false>(a, b, L, Ns, nfft, tw, ls);
        break;
      case 3: stage<R, 3, false>(a, b, L, Ns, nfft, tw, ls); break;
      case 4:
        if (p2) stage<R, 4, true>(a, b, L, Ns, nfft, tw, ls);
        else stage<R, 4, false>(a, b, L, Ns, nfft, tw, ls);
        break;
      case 5: stage<R, 5, false>(a, b, L, Ns, nfft, tw, ls); break;
      default:
        if (p2) stage<R, 8, true>(a, b, L, Ns, nfft, tw, ls);
        else stage<R, 8, false>(a, b, L, Ns, nfft, tw, ls);
        break;
    }
    Ns *= rad[s];
    __syncthreads();
    C2<R>* t = a; a = b; b = t;
  }
  return a;
}

// exp(-2 pi i k / N) from the two-level table (k < N)
template <typename R>
__device__ inline C2<R> wN(const C2<R>* lo, const C2<R>* hi, int64_t k) {
  return cm(lo[k & 1023], hi[k >> 10]);
}

constexpr int kCB = 16;        // columns per pass-1 workgroup (fewer for long columns)
constexpr int kP2MaxPairs = 16;   // row pairs per pass-2 workgroup, at most

template <typename R>
// cb columns per workgroup (cb lanes move one row segment), each column n1 + 1 elements apart
// in LDS: an odd stride puts the cb lanes of a segment on different bank pairs
__global__ __launch_bounds__(kFT) void k_pass1(FftPlanDev p, C2<R>* data, const int32_t* skip, int cb) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int n1 = p.n1, n2 = p.n2, ls = n1 + 1;
  C2<R>* a = (C2<R>*)smem;
  C2<R>* b = a + cb * ls;
  const int64_t row = blockIdx.y;
  if (skip && skip[row / 3] != 0) return;   // a faulted template's rows are not needed
  const int j2_0 = blockIdx.x * cb;
  C2<R>* z = data + row * p.n;
  const UDiv cbd(cb);
  // kU loads per thread in flight before their LDS stores, and kU twiddle pairs before the
  // multiplies and stores of the output loop
  constexpr int kU = 8;
  for (int i0 = threadIdx.x; i0 < cb * n1; i0 += kU * kFT) {
    C2<R> v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int i = i0 + u * kFT, j1 = cbd.div(i), j2 = j2_0 + (i - j1 * cb);
      v[u] = (i < cb * n1 && j2 < n2) ? z[(int64_t)j1 * n2 + j2] : C2<R>{(R)0, (R)0};
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int i = i0 + u * kFT, j1 = cbd.div(i), jj = i - j1 * cb;
      if (i < cb * n1) a[jj * ls + j1] = v[u];
    }
  }
  __syncthreads();
  const C2<R>* tw = (const C2<R>*)tw_ptr<R>(p.tw1d, p.tw1f);
  C2<R>* res = lds_fft<R>(a, b, n1, p.rad1, p.nr1, cb, tw, ls);
  const C2<R>* lo = (const C2<R>*)tw_ptr<R>(p.wlod, p.wlof);
  const C2<R>* hi = (const C2<R>*)tw_ptr<R>(p.whid, p.whif);
  for (int i0 = threadIdx.x; i0 < cb * n1; i0 += kU * kFT) {
    C2<R> lk[kU], hk[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int i = i0 + u * kFT, k1 = cbd.div(i), j2 = j2_0 + (i - k1 * cb);
      const bool on = i < cb * n1 && j2 < n2;
      const int64_t k = 2 * (int64_t)j2 * k1;           // 2 j2 k1 < 2n
      lk[u] = on ? lo[k & 1023] : C2<R>{(R)0, (R)0};
      hk[u] = on ? hi[k >> 10] : C2<R>{(R)0, (R)0};
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int i = i0 + u * kFT, k1 = cbd.div(i), jj = i - k1 * cb, j2 = j2_0 + jj;
      if (i < cb * n1 && j2 < n2) z[(int64_t)k1 * n2 + j2] = cm(res[jj * ls + k1], cm(lk[u], hk[u]));
    }
  }
}

// pass 2: np row pairs per workgroup, pairs p = np * blockIdx.x + q, q < np; pair p holds rows
// k1 = p and k1' = (n1 - p) mod n1 (slots 2q and 2q + 1; -1 where absent or a duplicate, the
// slot then transformed as zeros), which hold every mirror bin of each other
template <typename R>
__global__ __launch_bounds__(kFT) void k_pass2(FftPlanDev p, const C2<R>* data, int mode, double dt,
                                               C2<R>* spec, const double* wperm, int64_t ch_rows,
                                               double* partial, int64_t kb_lo, int64_t kb_hi,
                                               const int32_t* skip, int np) {
  if (skip && skip[blockIdx.y / 3] != 0) return;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[kFT / 64];
  __shared__ int rowk1[2 * kP2MaxPairs];
  const int n1 = p.n1, n2 = p.n2, nr = 2 * np;
  const int64_t n = p.n;
  const int pa = np * blockIdx.x;
  const int64_t row = blockIdx.y;
  if (threadIdx.x < np) {
    const int q = threadIdx.x, x = pa + q, y = (n1 - x) % n1;
    rowk1[2 * q] = x <= n1 / 2 ? x : -1;
    rowk1[2 * q + 1] = (x <= n1 / 2 && y != x) ? y : -1;
  }
  __syncthreads();
  C2<R>* a = (C2<R>*)smem;
  C2<R>* b = a + nr * n2;
  const C2<R>* z = data + row * n;
  const UDiv n2d(n2);
  {
    // kU loads per thread issued before their LDS stores (one memory latency per kU * kFT)
    constexpr int kU = 8;
    for (int i0 = threadIdx.x; i0 < nr * n2; i0 += kU * kFT) {
      C2<R> v[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int i = i0 + u * kFT;
        v[u] = C2<R>{(R)0, (R)0};
        if (i < nr * n2) {
          const int r = n2d.div(i), j2 = i - r * n2;
          const int k1 = rowk1[r];
          if (k1 >= 0) v[u] = z[(int64_t)k1 * n2 + j2];
        }
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int i = i0 + u * kFT;
        if (i < nr * n2) a[i] = v[u];
      }
    }
  }
  __syncthreads();
  const C2<R>* tw = (const C2<R>*)tw_ptr<R>(p.tw2d, p.tw2f);
  C2<R>* Z = lds_fft<R>(a, b, n2, p.rad2, p.nr2, nr, tw, n2);
  const C2<R>* lo = (const C2<R>*)tw_ptr<R>(p.wlod, p.wlof);
  const C2<R>* hi = (const C2<R>*)tw_ptr<R>(p.whid, p.whif);
  const double* w = wperm;
  double acc = 0.0;
  const int ch = (int)(row % 3);
  if (mode != 0) {
    // band power.  Bin k = k1 + n1 k2 lies in [kb_lo, kb_hi] only for k2 <= kb_hi / n1: the
    // items are (row slot r, k2) for k2 < K2, kU per thread with their weights and twiddles
    // loaded before they are used.  Weights are stored in pass-2 order (k1 n2 + k2; Nyquist n).
    const int64_t k2top = kb_hi / n1 < n2 - 1 ? kb_hi / n1 : n2 - 1;
    const int K2 = k2top > 0 ? (int)k2top + 1 : 1;
    const UDiv K2d(K2);
    const int nitem = nr * K2;
    constexpr int kU = 4;
    for (int i0 = threadIdx.x; i0 < nitem; i0 += kU * kFT) {
      bool on[kU];
      int rs[kU], k2s[kU];
      double wv[kU];
      C2<R> lk[kU], hk[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int i = i0 + u * kFT;
        const int r = K2d.div(i), k2 = i - r * K2;
        const int k1 = i < nitem ? rowk1[r] : -1;
        const int64_t k = k1 + (int64_t)n1 * k2;
        on[u] = k1 >= 0 && k >= kb_lo && k <= kb_hi;
        rs[u] = r;
        k2s[u] = k2;
        wv[u] = on[u] ? w[ch * (n + 1) + (int64_t)k1 * n2 + k2] : 0.0;
        lk[u] = on[u] ? lo[k & 1023] : C2<R>{(R)0, (R)0};
        hk[u] = on[u] ? hi[k >> 10] : C2<R>{(R)0, (R)0};
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        if (!on[u]) continue;
        const int r = rs[u], k2 = k2s[u], k1 = rowk1[r];
        const C2<R> Zk = Z[r * n2 + k2];
        C2<R> Zm;
        if (k1 == 0) {
          Zm = Z[r * n2 + (k2 == 0 ? 0 : n2 - k2)];
        } else {
          const int rm = (rowk1[r ^ 1] >= 0) ? (r ^ 1) : r;   // the mirror row sits in the paired slot
          Zm = Z[rm * n2 + (n2 - 1 - k2)];
        }
        const C2<R> zc = {Zm.x, -Zm.y};
        const C2<R> sm = sc(Zk + zc, (R)0.5), df = sc(Zk - zc, (R)0.5);
        const C2<R> X = sm + mi(cm(cm(lk[u], hk[u]), df));
        const double xr = (double)X.x, xi = (double)X.y;
        acc += wv[u] * (xr * xr + xi * xi);
      }
    }
    if (pa == 0 && threadIdx.x == 0 && n >= kb_lo && n <= kb_hi) {
      // Nyquist: Z_n = Z_0, twiddle -1
      const C2<R> Zk = Z[0], zc = {Z[0].x, -Z[0].y};
      const C2<R> sm = sc(Zk + zc, (R)0.5), df = sc(Zk - zc, (R)0.5);
      const C2<R> X = sm + mi(cm(C2<R>{(R)-1, (R)0}, df));
      const double xr = (double)X.x, xi = (double)X.y;
      acc += w[ch * (n + 1) + n] * (xr * xr + xi * xi);
    }
  }
  // full spectrum (mode 0): every k in the rows of this block, plus the Nyquist bin for pair 0
  const int nout = nr * n2 + (pa == 0 ? 1 : 0);
  for (int i = threadIdx.x; mode == 0 && i < nout; i += kFT) {
    int64_t k;
    C2<R> Zk, Zm;
    if (i < nr * n2) {
      const int r = n2d.div(i), k2 = i - r * n2;
      const int k1 = rowk1[r];
      if (k1 < 0) continue;
      k = k1 + (int64_t)n1 * k2;
      Zk = Z[r * n2 + k2];
      if (k1 == 0) {
        Zm = Z[r * n2 + (k2 == 0 ? 0 : n2 - k2)];
      } else {
        const int rm = (rowk1[r ^ 1] >= 0) ? (r ^ 1) : r;   // the mirror row sits in the paired slot
        Zm = Z[rm * n2 + (n2 - 1 - k2)];
      }
    } else {
      k = n;          // Nyquist: Z_n = Z_0
      Zk = Z[0];
      Zm = Z[0];
    }
    C2<R> zc = {Zm.x, -Zm.y};
    C2<R> sm = sc(Zk + zc, (R)0.5), df = sc(Zk - zc, (R)0.5);
    C2<R> wk = (k == n) ? C2<R>{(R)-1, (R)0} : wN<R>(lo, hi, k);
    C2<R> X = sm + mi(cm(wk, df));
    spec[row * (n + 1) + k] = sc(X, (R)dt);
  }
  if (mode != 0) {
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int i = 0; i < kFT / 64; ++i) t += red[i];
      partial[row * (n1 / 2 + 1) + pa] = t;
      for (int q = 1; q < np; ++q)
        if (pa + q <= n1 / 2) partial[row * (n1 / 2 + 1) + pa + q] = 0.0;
    }
  }
}

// ---------------------------------------------------------------------------
// Compile-time plans for the hot size N = 2^20 (n = 2^19 = 512 x 1024).
// Each stage reads all its butterfly inputs into registers, synchronises,
// writes the outputs in Stockham order into the same LDS buffer, synchronises.
// LS: distance between consecutive transforms in buf (>= L; padding avoids LDS bank conflicts);
// NT: threads of the workgroup
// PSH: element i of a series sits at i + (i >> PSH) (one spare slot per 2^PSH elements; 0: no
// slots).  A stage with NS < 32 writes each lane's RAD outputs NS elements apart, the lanes
// RAD NS elements apart; without the slots, 8-byte elements 8 (or 16) apart fall on a few
// bank groups of the 32 LDS banks.
template <int PSH>
__device__ inline int lix(int i) {
  return PSH ? i + (i >> PSH) : i;
}

template <typename R, int L, int NFFT, int RAD, int NS, int LS = L, int NT = kFT, int PSH = 0>
__device__ inline void ct_stage(C2<R>* buf, const C2<R>* tw) {
  constexpr int M = L / RAD;
  constexpr int JOBS = NFFT * M;
  constexpr int PER = (JOBS + NT - 1) / NT;
  constexpr int STEP = L / (NS * RAD);
  C2<R> v[PER][RAD];
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int job = threadIdx.x + p * NT;
    if (JOBS % NT == 0 || job < JOBS) {
      const int f = job / M, j = job % M, k = j % NS;
      const C2<R>* src = buf + f * LS;
#pragma unroll
      for (int r = 0; r < RAD; ++r) {
        v[p][r] = src[lix<PSH>(j + r * M)];
        if (NS > 1 && r > 0) v[p][r] = cm(v[p][r], tw[r * k * STEP]);
      }
      dft<R, RAD>(v[p]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int job = threadIdx.x + p * NT;
    if (JOBS % NT == 0 || job < JOBS) {
      const int f = job / M, j = job % M, k = j % NS;
      C2<R>* dst = buf + f * LS;
      const int d0 = (j / NS) * NS * RAD + k;
#pragma unroll
      for (int r = 0; r < RAD; ++r) dst[lix<PSH>(d0 + r * NS)] = v[p][r];
    }
  }
  __syncthreads();
}

template <typename R, int L, int NFFT, int NS, int RAD, int... REST>
__device__ inline void ct_fft(C2<R>* buf, const C2<R>* tw) {
  ct_stage<R, L, NFFT, RAD, NS>(buf, tw);
  if constexpr (sizeof...(REST) > 0) ct_fft<R, L, NFFT, NS * RAD, REST...>(buf, tw);
}

template <typename R, int L, int LS, int NT, int PSH, int NFFT, int NS, int RAD, int... REST>
__device__ inline void ct_fft_strided(C2<R>* buf, const C2<R>* tw) {
  ct_stage<R, L, NFFT, RAD, NS, LS, NT, PSH>(buf, tw);
  if constexpr (sizeof...(REST) > 0) ct_fft_strided<R, L, LS, NT, PSH, NFFT, NS * RAD, REST...>(buf, tw);
}

// pass 1 for n1 = 512: CB columns (128 bytes of each row) per workgroup.  Column c
// sits at buf[c * LP], LP = N1 + N1 / 8 + 1 (the column with a spare slot per eight
// elements, plus one): the 16 lanes that move one 128-byte row segment then touch 16
// different bank pairs instead of one.
constexpr int kP1Pad = 512 / 8 + 1;
// bytes of each row per workgroup (64 and 256 ran 2.21 and 1.89 ms against 1.59 on the bench
// workload: narrower segments waste the memory bursts, wider ones leave one workgroup per CU)
constexpr int kP1Bytes = 128;
constexpr int kP1Threads = 512;   // 2 workgroups of 65.7 KB fit a CU: 16 waves
template <typename R>
__global__ __launch_bounds__(kP1Threads) void k_pass1_512(FftPlanDev p, C2<R>* data, const int32_t* skip) {
  constexpr int N1 = 512, N2 = 1024, CB = kP1Bytes / (int)sizeof(C2<R>), LP = N1 + kP1Pad;
  extern __shared__ __align__(16) unsigned char smem[];
  C2<R>* buf = (C2<R>*)smem;      // [CB][LP]
  const int64_t row = blockIdx.y;
  if (skip && skip[row / 3] != 0) return;   // a faulted template's rows are not needed
  const int j2_0 = blockIdx.x * CB;
  C2<R>* z = data + row * ((int64_t)N1 * N2);
  constexpr int PT = CB * N1 / kP1Threads;   // elements per thread
  {
    // every load issued before the first LDS store (one memory latency)
    C2<R> v[PT];
#pragma unroll
    for (int t = 0; t < PT; ++t) {
      const int i = threadIdx.x + t * kP1Threads, j1 = i / CB, jj = i % CB;
      v[t] = z[(int64_t)j1 * N2 + j2_0 + jj];
    }
#pragma unroll
    for (int t = 0; t < PT; ++t) {
      const int i = threadIdx.x + t * kP1Threads, j1 = i / CB, jj = i % CB;
      buf[jj * LP + lix<3>(j1)] = v[t];
    }
  }
  __syncthreads();
  const C2<R>* tw = (const C2<R>*)tw_ptr<R>(p.tw1d, p.tw1f);
  ct_fft_strided<R, N1, LP, kP1Threads, 3, CB, 1, 8, 8, 8>(buf, tw);
  const C2<R>* lo = (const C2<R>*)tw_ptr<R>(p.wlod, p.wlof);
  const C2<R>* hi = (const C2<R>*)tw_ptr<R>(p.whid, p.whif);
  // twiddle tables read for all of this thread's elements before the first product
  C2<R> tl[PT], th[PT];
#pragma unroll
  for (int t = 0; t < PT; ++t) {
    const int i = threadIdx.x + t * kP1Threads, k1 = i / CB, jj = i % CB;
    const int64_t m2 = 2 * (int64_t)(j2_0 + jj) * k1;
    tl[t] = lo[m2 & 1023];
    th[t] = hi[m2 >> 10];
  }
#pragma unroll
  for (int t = 0; t < PT; ++t) {
    const int i = threadIdx.x + t * kP1Threads, k1 = i / CB, jj = i % CB;
    z[(int64_t)k1 * N2 + j2_0 + jj] = cm(buf[jj * LP + lix<3>(k1)], cm(tl[t], th[t]));
  }
}

// pass 2 for n2 = 1024: NP row pairs (up to 2 NP rows) per workgroup, each row in LDS with
// spare slots (below) so that the Stockham stages' strided writes spread over the banks.
template <typename R, int NP>
__global__ __launch_bounds__(kFT) void k_pass2_1024(FftPlanDev p, const C2<R>* data, int mode, double dt,
                                                    C2<R>* spec, const double* wperm, double* partial,
                                                    int64_t kb_lo, int64_t kb_hi, const int32_t* skip) {
  const int64_t row = blockIdx.y;
  if (skip && skip[row / 3] != 0) return;
  constexpr int N1 = 512, N2 = 1024, NR = 2 * NP;
  // FP32: stages of radix 16, 8, 8 (three LDS round trips instead of four; a radix-16 butterfly
  // holds 16 complex values per lane), rows with a spare slot per 16 elements, so that the
  // first stage's writes (lanes 16 elements apart) and every other access of a 16-lane group
  // meet distinct bank pairs; FP64 (twice the registers per value): radix 4, 4, 8, 8, no slots
  constexpr bool R16 = sizeof(R) == 4;
  constexpr int PSH = R16 ? 4 : (sizeof(R) == 4 ? 3 : 0);
  constexpr int LS = R16 ? N2 + N2 / 16 : (sizeof(R) == 4 ? N2 + N2 / 8 + 1 : N2);
  constexpr int64_t n = (int64_t)N1 * N2;
  __shared__ C2<R> buf[NR * LS];
  __shared__ int rowk1[NR];
  __shared__ double red[kFT / 64];
  const int pa = NP * blockIdx.x;      // pairs pa .. pa + NP - 1 (pair index <= N1/2)
  const C2<R>* z = data + row * n;
  // row slots 2q: pa + q, 2q + 1: N1 - pa - q (-1 where absent or a duplicate)
  if (threadIdx.x < NP) {
    const int q = threadIdx.x, a = pa + q, b = (N1 - a) % N1;
    rowk1[2 * q] = a <= N1 / 2 ? a : -1;
    rowk1[2 * q + 1] = (a <= N1 / 2 && b != a) ? b : -1;
  }
  __syncthreads();
  {
    // every load of the four rows issued before the first LDS store (one memory latency)
    constexpr int PT = NR * N2 / kFT;
    C2<R> v[PT];
#pragma unroll
    for (int m = 0; m < PT; ++m) {
      const int i = threadIdx.x + m * kFT;
      const int k1 = rowk1[i / N2];
      v[m] = k1 >= 0 ? z[(int64_t)k1 * N2 + (i % N2)] : C2<R>{(R)0, (R)0};
    }
#pragma unroll
    for (int m = 0; m < PT; ++m) {
      const int i = threadIdx.x + m * kFT;
      buf[(i / N2) * LS + lix<PSH>(i % N2)] = v[m];
    }
  }
  __syncthreads();
  const C2<R>* tw = (const C2<R>*)tw_ptr<R>(p.tw2d, p.tw2f);
  if constexpr (R16)
    ct_fft_strided<R, N2, LS, kFT, PSH, NR, 1, 16, 8, 8>(buf, tw);
  else
    ct_fft_strided<R, N2, LS, kFT, PSH, NR, 1, 4, 4, 8, 8>(buf, tw);
  const C2<R>* lo = (const C2<R>*)tw_ptr<R>(p.wlod, p.wlof);
  const C2<R>* hi = (const C2<R>*)tw_ptr<R>(p.whid, p.whif);
  double acc = 0.0;
  const int64_t ch = row % 3;
  if (mode != 0) {
    // band power.  Bin k = k1 + N1 k2 lies in [kb_lo, kb_hi] only for k2 <= kb_hi / N1; a thread
    // takes k2 = threadIdx.x + kFT m0 in each of the four rows, with the weights and twiddles
    // of the four rows loaded together before they are used.  Per thread the bins are summed
    // row by row within each m0.
    const int k2max = kb_hi / N1 < N2 - 1 ? (int)(kb_hi / N1) : N2 - 1;
    for (int m0 = 0; m0 * kFT <= k2max; ++m0) {
      const int k2 = threadIdx.x + m0 * kFT;
      bool on[NR];
      double wv[NR];
      C2<R> lk[NR], hk[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const int k1 = rowk1[r];
        const int64_t k = k1 + (int64_t)N1 * k2;
        on[r] = k1 >= 0 && k2 < N2 && k >= kb_lo && k <= kb_hi;
        wv[r] = on[r] ? wperm[ch * (n + 1) + (int64_t)k1 * N2 + k2] : 0.0;
        lk[r] = on[r] ? lo[k & 1023] : C2<R>{(R)0, (R)0};
        hk[r] = on[r] ? hi[k >> 10] : C2<R>{(R)0, (R)0};
      }
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        if (!on[r]) continue;
        const int k1 = rowk1[r];
        const C2<R> Zk = buf[r * LS + lix<PSH>(k2)];
        C2<R> Zm;
        if (k1 == 0) {
          Zm = buf[r * LS + lix<PSH>((N2 - k2) % N2)];
        } else {
          const int rm = (rowk1[r ^ 1] >= 0) ? (r ^ 1) : r;   // the mirror row sits in the paired slot
          Zm = buf[rm * LS + lix<PSH>(N2 - 1 - k2)];
        }
        const C2<R> zc = {Zm.x, -Zm.y};
        const C2<R> sm = sc(Zk + zc, (R)0.5), df = sc(Zk - zc, (R)0.5);
        const C2<R> X = sm + mi(cm(cm(lk[r], hk[r]), df));
        const double xr = (double)X.x, xi = (double)X.y;
        acc += wv[r] * (xr * xr + xi * xi);
      }
    }
    if (pa == 0 && threadIdx.x == 0 && n >= kb_lo && n <= kb_hi) {
      // Nyquist: Z_n = Z_0, twiddle -1
      const C2<R> Zk = buf[0], zc = {buf[0].x, -buf[0].y};
      const C2<R> sm = sc(Zk + zc, (R)0.5), df = sc(Zk - zc, (R)0.5);
      const C2<R> X = sm + mi(cm(C2<R>{(R)-1, (R)0}, df));
      const double xr = (double)X.x, xi = (double)X.y;
      acc += wperm[ch * (n + 1) + n] * (xr * xr + xi * xi);
    }
  }
  // full spectrum (mode 0)
  for (int i = threadIdx.x; mode == 0 && i < NR * N2 + 1; i += kFT) {
    int64_t k;
    C2<R> Zk, Zm;
    int k1, k2;
    if (i < NR * N2) {
      const int r = i / N2;
      k2 = i % N2;
      k1 = rowk1[r];
      if (k1 < 0) continue;
      k = k1 + (int64_t)N1 * k2;
      Zk = buf[r * LS + lix<PSH>(k2)];
      if (k1 == 0) {
        Zm = buf[r * LS + lix<PSH>((N2 - k2) % N2)];
      } else {
        const int rm = (rowk1[r ^ 1] >= 0) ? (r ^ 1) : r;   // the mirror row sits in the paired slot
        Zm = buf[rm * LS + lix<PSH>(N2 - 1 - k2)];
      }
    } else {
      if (pa != 0) continue;
      k = n;            // Nyquist: Z_n = Z_0
      k1 = 0;
      k2 = 0;
      Zk = buf[0];
      Zm = buf[0];
    }
    C2<R> zc = {Zm.x, -Zm.y};
    C2<R> sm = sc(Zk + zc, (R)0.5), df = sc(Zk - zc, (R)0.5);
    C2<R> wk = (k == n) ? C2<R>{(R)-1, (R)0} : wN<R>(lo, hi, k);
    C2<R> X = sm + mi(cm(wk, df));
    spec[row * (n + 1) + k] = sc(X, (R)dt);
  }
  if (mode != 0) {
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int i = 0; i < kFT / 64; ++i) t += red[i];
      partial[row * (N1 / 2 + 1) + pa] = t;
      for (int q = 1; q < NP; ++q)
        if (pa + q <= N1 / 2) partial[row * (N1 / 2 + 1) + pa + q] = 0.0;
    }
  }
}

static bool hot_plan(const FftPlanDev& p) { return p.n1 == 512 && p.n2 == 1024; }
// row pairs per pass-2 workgroup (one pair, or four, ran 15 % and 30 % slower on the bench
// workload; ordering the rows channel by channel, so that concurrent workgroups share one
// channel's weights, changed nothing)
constexpr int kP2Pairs = 2;

template <typename R>
static hipError_t p1(const FftPlanDev& p, void* data, int64_t rows, const int32_t* skip, hipStream_t s) {
  if (hot_plan(p)) {
    constexpr int CB = kP1Bytes / (int)sizeof(C2<R>);
    const int bytes = CB * (512 + kP1Pad) * (int)sizeof(C2<R>);
    hipError_t e = hipFuncSetAttribute((const void*)k_pass1_512<R>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
    dim3 grid((unsigned)(p.n2 / CB), (unsigned)rows);
    hipLaunchKernelGGL(k_pass1_512<R>, grid, dim3(kP1Threads), bytes, s, p, (C2<R>*)data, skip);
    return hipGetLastError();
  }
  // kCB columns where that fits 64 KiB of LDS, else as many as fit 160 KiB
  int cb = kCB;
  if (2 * (size_t)cb * (p.n1 + 1) * sizeof(C2<R>) > 65536)
    while (cb > 1 && 2 * (size_t)cb * (p.n1 + 1) * sizeof(C2<R>) > 160 * 1024) cb /= 2;
  size_t bytes = 2 * (size_t)cb * (p.n1 + 1) * sizeof(C2<R>);
  hipError_t e = hipFuncSetAttribute((const void*)k_pass1<R>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  dim3 grid((unsigned)((p.n2 + cb - 1) / cb), (unsigned)rows);
  hipLaunchKernelGGL(k_pass1<R>, grid, dim3(kFT), bytes, s, p, (C2<R>*)data, skip, cb);
  return hipGetLastError();
}

hipError_t launch_fft_pass1(const FftPlanDev& p, void* data, int64_t rows, int precision, const int32_t* skip,
                            hipStream_t s) {
  return precision == 0 ? p1<double>(p, data, rows, skip, s) : p1<float>(p, data, rows, skip, s);
}

template <typename R>
static hipError_t p2(const FftPlanDev& p, const void* data, int64_t rows, int mode, double dt, void* spec,
                     const double* wperm, int64_t ch_rows, double* partial, int64_t kb_lo, int64_t kb_hi,
                     const int32_t* skip, hipStream_t s) {
  if (hot_plan(p)) {
    constexpr int NP = kP2Pairs;
    dim3 grid((unsigned)((p.n1 / 2 + NP) / NP), (unsigned)rows);
    hipLaunchKernelGGL((k_pass2_1024<R, NP>), grid, dim3(kFT), 0, s, p, (const C2<R>*)data, mode, dt, (C2<R>*)spec,
                       wperm, partial, kb_lo, kb_hi, skip);
    return hipGetLastError();
  }
  // pairs per workgroup: about 2048 elements of rows (two buffers), at most kP2MaxPairs
  int np = 1024 / p.n2;
  np = np < 1 ? 1 : (np > kP2MaxPairs ? kP2MaxPairs : np);
  size_t bytes = 2 * (size_t)(2 * np) * p.n2 * sizeof(C2<R>);
  hipError_t e = hipFuncSetAttribute((const void*)k_pass2<R>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  dim3 grid((unsigned)((p.n1 / 2 + np) / np), (unsigned)rows);
  hipLaunchKernelGGL(k_pass2<R>, grid, dim3(kFT), bytes, s, p, (const C2<R>*)data, mode, dt, (C2<R>*)spec, wperm,
                     ch_rows, partial, kb_lo, kb_hi, skip, np);
  return hipGetLastError();
}

hipError_t launch_fft_pass2(const FftPlanDev& p, const void* data, int64_t rows, int precision, int mode, double dt,
                            void* spec, const double* wperm, int64_t ch_rows, double* partial, int64_t kb_lo,
                            int64_t kb_hi, const int32_t* skip, hipStream_t s) {
  return precision == 0 ? p2<double>(p, data, rows, mode, dt, spec, wperm, ch_rows, partial, kb_lo, kb_hi, skip, s)
                        : p2<float>(p, data, rows, mode, dt, spec, wperm, ch_rows, partial, kb_lo, kb_hi, skip, s);
}

// weights in pass-2 order: w[c][k1 * n2 + k2] = 1/S_c(k) inside the band of an
// enabled channel, 0 elsewhere; w[c][n] for the Nyquist bin.
__global__ void k_weights(FftPlanDev p, const double* S0, const double* S1, const double* S2, int k_lo, int k_hi,
                          int channels, double* w) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int c = blockIdx.y;
  const int64_t n = p.n;
  if (i > n) return;
  int64_t k;
  if (i == n) k = n;
  else {
    int64_t k1 = i / p.n2, k2 = i - k1 * p.n2;
    k = k1 + (int64_t)p.n1 * k2;
  }
  const double* S = c == 0 ? S0 : (c == 1 ? S1 : S2);
  double v = 0.0;
  if ((channels >> c) & 1)
    if (k >= k_lo && k <= k_hi) v = 1.0 / S[k];
  w[c * (n + 1) + i] = v;
}

hipError_t launch_weights(const FftPlanDev& p, const double* const* S, int k_lo, int k_hi, int channels, double* w,
                          hipStream_t s) {
  dim3 grid((unsigned)((p.n + 1 + 255) / 256), 3);
  hipLaunchKernelGGL(k_weights, grid, dim3(256), 0, s, p, S[0], S[1], S[2], k_lo, k_hi, channels, w);
  return hipGetLastError();
}

// Error-free sum of two doubles (Knuth's TwoSum): a + b = s + e exactly.
__device__ inline void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// per template: sum over 3 channels x npairs partial sums in a fixed order.  Every step is
// compensated: each thread keeps a (sum, error) pair over its strided partials (TwoSum per
// term), and the pairs are merged by TwoSum through the wavefront and block tree, the errors
// added at the end.  A non-finite result marks the template with status 2 and logL = -inf.
__global__ __launch_bounds__(256) void k_finalize(const double* partial, int npairs, double scale, double dd,
                                                  int32_t* status, double* logl, double* logl_full,
                                                  double* inner) {
  __shared__ double red[4], rede[4];
  const int64_t b = blockIdx.x;
  const double* q = partial + b * 3 * npairs;
  const int total = 3 * npairs;
  double cs = 0.0, ce = 0.0;
  for (int i = threadIdx.x; i < total; i += 256) {
    double e;
    two_sum(cs, q[i], cs, e);
    ce += e;
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double os = __shfl_down(cs, off, 64), oe = __shfl_down(ce, off, 64);
    double e;
    two_sum(cs, os, cs, e);
    ce += oe + e;
  }
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = cs;
    rede[threadIdx.x >> 6] = ce;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double s = red[0], se = rede[0];
  for (int i = 1; i < 4; ++i) {
    double e;
    two_sum(s, red[i], s, e);
    se += rede[i] + e;
  }
  const double rr = scale * (s + se);
  if (inner) inner[b] = rr;
  const bool bad = status && status[b] != 0;
  double full = bad ? -INFINITY : -0.5 * rr;
  if (!bad && !isfinite(full)) {
    full = -INFINITY;
    if (status) status[b] = 2;
  }
  if (logl_full) logl_full[b] = full;
  if (logl) logl[b] = full + 0.5 * dd;
}

hipError_t launch_finalize(const double* partial, int64_t batch, int npairs, double scale, double dd,
                           int32_t* status, double* logl, double* logl_full, double* inner, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3((unsigned)batch), dim3(256), 0, s, partial, npairs, scale, dd, status, logl,
                     logl_full, inner);
  return hipGetLastError();
}

}  // namespace lt
