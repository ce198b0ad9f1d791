// liblisatd host side: context, validation, FFT plans, orbit node tables, TDI
// term tables and the extern "C" entry points declared in include/lisatd.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/lisatd.h"
#include "lt_kernels.hpp"

using namespace lt;

static thread_local std::string g_err;

namespace lt {
void set_error(const std::string& msg) { g_err = msg; }
}  // namespace lt

static lt_status fail(lt_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define LT_HIP(call)                                                                 \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail(LT_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// ------------------------------------------------------------------ buffers
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t ensure(size_t b) {
    if (b <= bytes) return hipSuccess;
    if (p) {
      // kernels of earlier calls (on either of the context's streams) may still read it
      hipError_t e = hipDeviceSynchronize();
      if (e != hipSuccess) return e;
      e = hipFree(p);
      if (e != hipSuccess) return e;
      p = nullptr;
      bytes = 0;
    }
    hipError_t e = hipMalloc(&p, b);
    if (e == hipSuccess) bytes = b;
    return e;
  }
};

struct Plan {
  FftPlanDev dev{};
  DevBuf tw1d, tw1f, tw2d, tw2f, wlod, wlof, whid, whif;
};

struct OrbitTab {
  DevBuf tab;
  OrbitDev dev{};
};

struct lt_ctx {
  int device = 0;
  std::map<int64_t, std::unique_ptr<Plan>> plans;
  std::map<std::tuple<int, double, double, double, double, double, double, int64_t, uint64_t>,
           std::unique_ptr<OrbitTab>>
      orbits;
  DevBuf tpl, work, partial, wperm, wave, nodes, refs;
  DevBuf ws;              // lt_tdi_loglike's scratch when the caller passes no workspace
  DevBuf tune_out;        // lt_autotune's logL outputs
  lt_tuning tune{256, 1, 0, 4};   // launch shape of the likelihood (lt_ctx_set_tuning, lt_autotune)
  int tune_discarded = 0;         // shapes lt_autotune found to change a result (none expected)
  void* scratch = nullptr;   // this device's copy of the fixed scratch (lt_tdi_loglike_noalloc)
  bool profiling = false;
  struct Rec { int cls; hipEvent_t a, b; };
  std::vector<Rec> recs;
  double prof_ms[8] = {0};
  int64_t prof_n[8] = {0};
};

// ------------------------------------------------------------------ fixed scratch
// Device memory of lt_tdi_loglike_noalloc, for callers that cannot allocate: one copy per GPU,
// loaded with the library and held until the process ends.  In host code the array's name is
// not a device address: every host use goes through the address hipGetSymbolAddress returns for
// the current device (kept per device by lt_ctx_create).  Calls on one GPU share it.
constexpr size_t kFixedScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[kFixedScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mutex;
static void* g_scratch_ptr[kMaxDevices];

// the fixed scratch's device address on `device` (current): looked up once per device
static hipError_t fixed_scratch(int device, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

// Events bracket a launch on its stream when profiling is on.
struct Prof {
  lt_ctx* c;
  int cls;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  Prof(lt_ctx* c_, int cls_, hipStream_t s_) : c(c_), cls(cls_), s(s_) {
    if (c->profiling) {
      (void)hipEventCreate(&a);
      (void)hipEventCreate(&b);
      (void)hipEventRecord(a, s);
    }
  }
  ~Prof() {
    if (c->profiling) {
      (void)hipEventRecord(b, s);
      c->recs.push_back({cls, a, b});
    }
  }
};

static void drain_profile(lt_ctx* c) {
  for (auto& r : c->recs) {
    (void)hipEventSynchronize(r.b);
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      c->prof_ms[r.cls] += ms;
      c->prof_n[r.cls] += 1;
    }
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  c->recs.clear();
}

// ------------------------------------------------------------------ FFT plan
static bool radices(int L, int* rad, int* nr) {
  int k = 0;
  while (L % 5 == 0) { rad[k++] = 5; L /= 5; }
  while (L % 3 == 0) { rad[k++] = 3; L /= 3; }
  int a = 0;
  while (L % 2 == 0) { ++a; L /= 2; }
  if (L != 1) return false;
  int p = a / 3, r = a % 3;
  if (r == 1 && p >= 1) { p -= 1; rad[k++] = 4; rad[k++] = 4; }
  else if (r == 1) rad[k++] = 2;
  else if (r == 2) rad[k++] = 4;
  for (int i = 0; i < p; ++i) rad[k++] = 8;
  if (k > 12) return false;
  *nr = k;
  return true;
}

static void host_tw(std::vector<double>& d, int64_t count, int64_t stride, int64_t N) {
  d.resize(2 * count);
  for (int64_t k = 0; k < count; ++k) {
    int64_t m = (k * stride) % N;
    double ang = -2.0 * M_PI * (double)m / (double)N;
    d[2 * k] = std::cos(ang);
    d[2 * k + 1] = std::sin(ang);
  }
}

static hipError_t upload(DevBuf& dd, DevBuf& df, const std::vector<double>& h) {
  hipError_t e = dd.ensure(h.size() * sizeof(double));
  if (e != hipSuccess) return e;
  e = df.ensure(h.size() * sizeof(float));
  if (e != hipSuccess) return e;
  std::vector<float> f(h.begin(), h.end());
  e = hipMemcpy(dd.p, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  return hipMemcpy(df.p, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice);
}

// n = N/2 = n1 * n2 with n1 even, both <= 1024 and built from the supported radices, the two
// factors as close as possible (false when no such split exists)
static bool plan_shape(int64_t N, int* n1, int* n2) {
  if (N < 8 || N % 2 != 0) return false;
  int64_t n = N / 2;
  int best1 = -1, best2 = -1;
  double bestscore = 1e300;
  for (int64_t d = 2; d <= 1024; d += 2) {
    if (n % d) continue;
    int64_t e = n / d;
    if (e > 1024 || e < 1) continue;
    int r[12], nr;
    if (!radices((int)d, r, &nr) || !radices((int)e, r, &nr)) continue;
    double score = std::fabs(std::log((double)d) - std::log((double)e)) + (e < d ? 1e-3 : 0.0);
    if (score < bestscore) { bestscore = score; best1 = (int)d; best2 = (int)e; }
  }
  *n1 = best1;
  *n2 = best2;
  return best1 > 0;
}

// The context's FFT plan for length N, built and uploaded on first use (may_alloc false: only
// an existing plan, LT_ERR_CONFIG otherwise)
static lt_status get_plan(lt_ctx* c, int64_t N, Plan** out, bool may_alloc = true) {
  auto it = c->plans.find(N);
  if (it != c->plans.end()) {
    *out = it->second.get();
    return LT_OK;
  }
  if (N < 8 || N % 2 != 0) return fail(LT_ERR_SHAPE, "FFT length must be even and >= 8");
  int64_t n = N / 2;
  int best1, best2;
  if (!plan_shape(N, &best1, &best2))
    return fail(LT_ERR_UNSUPPORTED, "N/2 must factor as n1*n2 (n1 even, both <= 1024) over radices 2,3,5");
  if (!may_alloc)
    return fail(LT_ERR_CONFIG, "no FFT plan for this grid length in the context (a call that may allocate builds it)");
  auto p = std::make_unique<Plan>();
  FftPlanDev& d = p->dev;
  d.N = N;
  d.n = n;
  d.n1 = best1;
  d.n2 = best2;
  radices(d.n1, d.rad1, &d.nr1);
  radices(d.n2, d.rad2, &d.nr2);
  std::vector<double> h;
  host_tw(h, d.n1, 1, d.n1);
  LT_HIP(upload(p->tw1d, p->tw1f, h));
  host_tw(h, d.n2, 1, d.n2);
  LT_HIP(upload(p->tw2d, p->tw2f, h));
  host_tw(h, 1024, 1, N);
  LT_HIP(upload(p->wlod, p->wlof, h));
  host_tw(h, N / 1024 + 2, 1024, N);
  LT_HIP(upload(p->whid, p->whif, h));
  d.tw1d = (const double*)p->tw1d.p; d.tw1f = (const float*)p->tw1f.p;
  d.tw2d = (const double*)p->tw2d.p; d.tw2f = (const float*)p->tw2f.p;
  d.wlod = (const double*)p->wlod.p; d.wlof = (const float*)p->wlof.p;
  d.whid = (const double*)p->whid.p; d.whif = (const float*)p->whif.p;
  *out = p.get();
  c->plans[N] = std::move(p);
  return LT_OK;
}

// ------------------------------------------------------------------ orbits
static const int kLinkLabel[6] = {1, 2, 3, -1, -2, -3};

static void link_ends(int l, int* s, int* r) {
  int k = l > 0 ? l : -l;
  int a = (k + 1) % 3 + 1, b = k % 3 + 1;
  if (l > 0) { *s = a; *r = b; } else { *s = b; *r = a; }
}

// four-point Lagrange weights of a uniform table at time t: samples j0 .. j0 + 3 around t
// (false outside the table)
static bool tab_weights(const lt_orbit& o, double t, int64_t* j0, double* w) {
  const double x = (t - o.tab_t0) / o.tab_dt;
  const double fj = std::floor(x);
  if (!(fj >= 1.0 && fj + 2.0 <= (double)(o.n_tab - 1))) return false;
  const double f = x - fj;
  const double fm1 = f - 1.0, fm2 = f - 2.0, fp1 = f + 1.0;
  w[0] = -f * fm1 * fm2 * (1.0 / 6.0);
  w[1] = fp1 * fm1 * fm2 * 0.5;
  w[2] = -fp1 * f * fm2 * 0.5;
  w[3] = fp1 * f * fm1 * (1.0 / 6.0);
  *j0 = (int64_t)fj - 1;
  return true;
}

// interpolated table column: v[(j) * stride + col]
static double tab_value(const lt_orbit& o, const double* v, int stride, int col, double t) {
  int64_t j0 = 0;
  double w[4];
  tab_weights(o, t, &j0, w);   // coverage checked before any evaluation
  double a = 0.0;
  for (int m = 0; m < 4; ++m) a += w[m] * v[(j0 + m) * stride + col];
  return a;
}

static void sc_position(const lt_orbit& o, int k, double t, double* r) {
  if (o.kind == LT_ORBIT_TABLE) {
    for (int q = 0; q < 3; ++q) r[q] = tab_value(o, o.pos, 9, (k - 1) * 3 + q, t);
    return;
  }
  const double sig = 2.0 * M_PI * (k - 1) / 3.0;
  if (o.kind == LT_ORBIT_STATIC_EQUAL) {
    const double rho = o.arm_m / std::sqrt(3.0);
    const double cs = std::cos(sig), sn = std::sin(sig);
    r[0] = o.au_m + rho * cs * 0.5;
    r[1] = rho * sn;
    r[2] = rho * cs * (std::sqrt(3.0) / 2.0);
    return;
  }
  const double e = o.arm_m / (2.0 * std::sqrt(3.0) * o.au_m);
  const double inc = std::sqrt(3.0) * e;
  const double Om = 2.0 * M_PI / kYear;
  const double M = Om * (t - o.t_ref) + o.phase0 - sig;
  double E = M;
  for (int i = 0; i < 50; ++i) {
    double dE = (E - e * std::sin(E) - M) / (1.0 - e * std::cos(E));
    E -= dE;
    if (std::fabs(dE) < 1e-17) break;
  }
  const double xo = o.au_m * (std::cos(E) - e);
  const double yo = o.au_m * std::sqrt(1.0 - e * e) * std::sin(E);
  const double x1 = xo * std::cos(inc), z1 = xo * std::sin(inc);
  const double cs = std::cos(sig), sn = std::sin(sig);
  r[0] = cs * x1 - sn * yo;
  r[1] = sn * x1 + cs * yo;
  r[2] = z1;
}

static double light_time(const lt_orbit& o, int l, double t, double* rr, double* rs) {
  int s, r;
  link_ends(l, &s, &r);
  sc_position(o, r, t, rr);
  if (o.kind == LT_ORBIT_TABLE) {
    const int li = l > 0 ? l - 1 : 2 - l;   // column of link l: 1, 2, 3, -1, -2, -3
    const double L = tab_value(o, o.ltt, 6, li, t);
    sc_position(o, s, t - L, rs);
    return L;
  }
  if (o.kind == LT_ORBIT_STATIC_EQUAL) {
    sc_position(o, s, t, rs);
    return o.arm_m / kC;
  }
  sc_position(o, s, t, rs);
  double L = std::sqrt((rr[0] - rs[0]) * (rr[0] - rs[0]) + (rr[1] - rs[1]) * (rr[1] - rs[1]) +
                       (rr[2] - rs[2]) * (rr[2] - rs[2])) / kC;
  for (int i = 0; i < 20; ++i) {
    sc_position(o, s, t - L, rs);
    double Ln = std::sqrt((rr[0] - rs[0]) * (rr[0] - rs[0]) + (rr[1] - rs[1]) * (rr[1] - rs[1]) +
                          (rr[2] - rs[2]) * (rr[2] - rs[2])) / kC;
    bool done = std::fabs(Ln - L) < 1e-15;
    L = Ln;
    if (done) break;
  }
  sc_position(o, s, t - L, rs);
  return L;
}

static constexpr int kNodeSpacing = 256;
static constexpr int kNodeJ0 = 2;

// FNV-1a over the bytes of a table orbit's arrays (0 for the analytic kinds)
static uint64_t orbit_hash(const lt_orbit* o) {
  if (o->kind != LT_ORBIT_TABLE) return 0;
  uint64_t h = 1469598103934665603ull;
  auto mix = [&h](const void* p, size_t n) {
    const unsigned char* b = (const unsigned char*)p;
    for (size_t i = 0; i < n; ++i) {
      h ^= b[i];
      h *= 1099511628211ull;
    }
  };
  mix(&o->n_tab, sizeof(o->n_tab));
  mix(&o->tab_t0, sizeof(double));
  mix(&o->tab_dt, sizeof(double));
  mix(o->pos, (size_t)o->n_tab * 9 * sizeof(double));
  mix(o->ltt, (size_t)o->n_tab * 6 * sizeof(double));
  return h;
}

// orbit nodes of a grid: every tile's nodes, one interval and the j0 offset on each side
static int orbit_node_count(const lt_grid* g) {
  const int64_t ntile = (g->n + tdi_tile() - 1) / tdi_tile();
  const int64_t last = ntile * tdi_tile() - 1;
  return (int)(last / kNodeSpacing + 3 + kNodeJ0 + 2);
}

// The context's orbit node table for (orbit, grid), built on the host and uploaded on first use
// (may_alloc false: only an existing table, LT_ERR_CONFIG otherwise)
static lt_status get_orbit(lt_ctx* c, const lt_orbit* o, const lt_grid* g, OrbitDev* out, bool may_alloc = true) {
  auto key = std::make_tuple(o->kind, o->arm_m, o->au_m, o->phase0, o->t_ref, g->t0, g->dt, (int64_t)g->n,
                             orbit_hash(o));
  auto it = c->orbits.find(key);
  if (it != c->orbits.end()) {
    *out = it->second->dev;
    return LT_OK;
  }
  if (!may_alloc)
    return fail(LT_ERR_CONFIG, "no node table for this orbit and grid in the context (a call that may allocate builds it)");
  const int n_nodes = orbit_node_count(g);
  if (o->kind == LT_ORBIT_TABLE) {
    // every node time, and every emission time up to the longest light time before it
    double maxL = 0.0;
    for (int64_t j = 0; j < o->n_tab * 6; ++j) maxL = std::fmax(maxL, o->ltt[j]);
    const double t_lo = g->t0 + (double)((int64_t)(0 - kNodeJ0) * kNodeSpacing) * g->dt - maxL;
    const double t_hi = g->t0 + (double)((int64_t)(n_nodes - 1 - kNodeJ0) * kNodeSpacing) * g->dt;
    int64_t j0;
    double w[4];
    if (!tab_weights(*o, t_lo, &j0, w) || !tab_weights(*o, t_hi, &j0, w))
      return fail(LT_ERR_CONFIG, "orbit table does not cover the grid (nodes, light times and one interval)");
  }
  std::vector<double> tab((size_t)n_nodes * kNodeStride);
  double maxL = 0.0;
  for (int j = 0; j < n_nodes; ++j) {
    double t = g->t0 + (double)((int64_t)(j - kNodeJ0) * kNodeSpacing) * g->dt;
    for (int li = 0; li < 6; ++li) {
      double rr[3], rs[3];
      double L = light_time(*o, kLinkLabel[li], t, rr, rs);
      double d[3] = {rr[0] - rs[0], rr[1] - rs[1], rr[2] - rs[2]};
      double nn = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      double* e = tab.data() + (size_t)j * kNodeStride + li * kNodeLink;
      e[0] = L;
      for (int q = 0; q < 3; ++q) {
        e[1 + q] = rr[q] / kC;
        e[4 + q] = rs[q] / kC;
        e[7 + q] = d[q] / nn;
      }
      maxL = std::fmax(maxL, L);
    }
  }
  auto ot = std::make_unique<OrbitTab>();
  LT_HIP(ot->tab.ensure(tab.size() * sizeof(double)));
  LT_HIP(hipMemcpy(ot->tab.p, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice));
  ot->dev.tab = (const double*)ot->tab.p;
  ot->dev.n_nodes = n_nodes;
  ot->dev.j0 = kNodeJ0;
  ot->dev.spacing = kNodeSpacing;
  ot->dev.max_light_time = maxL;
  *out = ot->dev;
  c->orbits[key] = std::move(ot);
  return LT_OK;
}

// ------------------------------------------------------------ TDI term tables
struct HostTerm { int sign, link; std::vector<int> delays; };

// Michelson X: Eq. (2.9) (generation 1.5) and Eq. (2.10) (generation 2.0, with
// the eleventh delay read as 2L-2 + L2 + 2L3 + 2L-3).
static std::vector<HostTerm> x_terms(int gen) {
  std::vector<HostTerm> v = {{+1, -3, {3, 2, -2}}, {-1, -3, {3}}};
  if (gen == 20) {
    v.push_back({+1, -3, {-2, 2, 3, 3, -3}});
    v.push_back({-1, -3, {3, 3, -3, -2, -2, 2, 2}});
  }
  v.push_back({+1, 3, {2, -2}});
  v.push_back({-1, 3, {}});
  if (gen == 20) {
    v.push_back({+1, 3, {-2, 2, 3, -3}});
    v.push_back({-1, 3, {3, -3, -2, -2, 2, 2}});
  }
  v.push_back({+1, 2, {-2}});
  v.push_back({-1, 2, {-2, -3, 3}});
  if (gen == 20) {
    v.push_back({+1, 2, {-2, -2, 2, 3, 3, -3, -3}});
    v.push_back({-1, 2, {3, -3, -2, -2, 2}});
  }
  v.push_back({+1, -2, {}});
  v.push_back({-1, -2, {-3, 3}});
  if (gen == 20) {
    v.push_back({+1, -2, {-2, 2, 3, 3, -3, -3}});
    v.push_back({-1, -2, {3, -3, -2, 2}});
  }
  return v;
}

static int rot_label(int l, int times) {
  int s = l > 0 ? 1 : -1, k = l > 0 ? l : -l;
  for (int i = 0; i < times; ++i) k = k % 3 + 1;
  return s * k;
}

static int link_index(int l) {
  for (int i = 0; i < 6; ++i)
    if (kLinkLabel[i] == l) return i;
  return -1;
}

static TermTable make_terms(int gen) {
  TermTable T;
  std::memset(&T, 0, sizeof(T));
  auto xs = x_terms(gen);
  for (int ch = 0; ch < 3; ++ch) {
    T.n_terms[ch] = (int)xs.size();
    for (size_t i = 0; i < xs.size(); ++i) {
      Term& t = T.t[ch][i];
      t.sign = xs[i].sign;
      t.link = link_index(rot_label(xs[i].link, ch));
      int cnt[6] = {0, 0, 0, 0, 0, 0};
      for (int d : xs[i].delays) cnt[link_index(rot_label(d, ch))] += 1;
      t.nd = 0;
      for (int li = 0; li < 6; ++li)
        if (cnt[li]) {
          t.dlink[t.nd] = li;
          t.dcnt[t.nd] = cnt[li];
          ++t.nd;
        }
      int total = 0;
      for (int li = 0; li < 6; ++li) total += cnt[li];
      if (total > T.max_delays) T.max_delays = total;
    }
    for (int i = 0; i < T.n_terms[ch]; ++i) {
      const int link = T.t[ch][i].link;
      int g = 0;
      while (g < T.n_groups[ch] && T.g_link[ch][g] != link) ++g;
      if (g == T.n_groups[ch]) {
        T.g_link[ch][g] = link;
        T.g_n[ch][g] = 0;
        ++T.n_groups[ch];
      }
      T.g_t[ch][g][T.g_n[ch][g]++] = i;
    }
    for (int g = 0; g < T.n_groups[ch]; ++g) {
      int lo = 1 << 20, hi = 0;
      for (int q = 0; q < T.g_n[ch][g]; ++q) {
        const Term& t = T.t[ch][T.g_t[ch][g][q]];
        int total = 0;
        for (int k = 0; k < t.nd; ++k) total += t.dcnt[k];
        lo = std::min(lo, total);
        hi = std::max(hi, total);
      }
      T.g_span = std::max(T.g_span, (double)(hi - lo) + 0.05 * lo);
    }
  }
  return T;
}

// ------------------------------------------------------------------ checks
// templates per launch of lt_tdi_loglike (lt_tuning.chunk, 256 by default): bounds the
// workspace (2 waveform + 3 TDI series of n samples per template) and amortises the
// per-launch tables and the launch tails

static lt_status check_common(lt_ctx* c, const double* params, int64_t batch, const lt_wf_cfg* cfg, const lt_grid* g) {
  if (!c) return fail(LT_ERR_NULL, "null context");
  if (!params) return fail(LT_ERR_NULL, "null params");
  if (!cfg || !g) return fail(LT_ERR_NULL, "null config or grid");
  if (batch < 1 || batch > 65535) return fail(LT_ERR_SHAPE, "batch must be in [1, 65535]");
  if (g->n < 8 || g->n > ((int64_t)1 << 26)) return fail(LT_ERR_SHAPE, "grid n must be in [8, 2^26]");
  if (!(g->dt > 0.0) || !std::isfinite(g->t0)) return fail(LT_ERR_SHAPE, "bad grid t0 / dt");
  if (cfg->mode_mask <= 0 || cfg->mode_mask > 31) return fail(LT_ERR_CONFIG, "mode_mask must be a nonzero subset of 31");
  if (cfg->precessing != 0 && cfg->precessing != 1) return fail(LT_ERR_CONFIG, "precessing must be 0 or 1");
  if (cfg->precision != LT_FP64 && cfg->precision != LT_MIXED) return fail(LT_ERR_CONFIG, "bad precision");
  if (!(cfg->f_low > 0.0) || !(cfg->f_ref > 0.0)) return fail(LT_ERR_CONFIG, "f_low and f_ref must be positive");
  if (cfg->coarse < 0 || cfg->coarse > 2) return fail(LT_ERR_CONFIG, "coarse must be 0, 1 or 2");
  LT_HIP(hipSetDevice(c->device));
  return LT_OK;
}

static lt_status check_tdi(const lt_orbit* o, const lt_tdi_cfg* t, const lt_grid* g) {
  if (!o || !t) return fail(LT_ERR_NULL, "null orbit or tdi config");
  if (o->kind != LT_ORBIT_STATIC_EQUAL && o->kind != LT_ORBIT_KEPLER && o->kind != LT_ORBIT_TABLE)
    return fail(LT_ERR_UNSUPPORTED, "orbit kind");
  if (o->kind == LT_ORBIT_TABLE) {
    if (!o->pos || !o->ltt) return fail(LT_ERR_NULL, "orbit table arrays");
    if (o->n_tab < 4 || !(o->tab_dt > 0.0) || !std::isfinite(o->tab_t0)) return fail(LT_ERR_CONFIG, "orbit table grid");
    if (!(o->arm_m > 0.0)) return fail(LT_ERR_CONFIG, "bad arm");
    for (int64_t j = 0; j < o->n_tab * 6; ++j)
      if (!(o->ltt[j] > 0.0 && o->ltt[j] <= 1.01 * o->arm_m / kC))
        return fail(LT_ERR_CONFIG, "orbit table light times must lie in (0, 1.01 arm_m / c]");
    for (int64_t j = 0; j < o->n_tab * 9; ++j)
      if (!std::isfinite(o->pos[j])) return fail(LT_ERR_CONFIG, "orbit table positions must be finite");
  } else if (!(o->arm_m > 0.0) || !(o->au_m > 0.0) || o->arm_m > 0.1 * o->au_m) {
    return fail(LT_ERR_CONFIG, "bad arm / au");
  }
  if (t->generation != 15 && t->generation != 20) return fail(LT_ERR_CONFIG, "generation must be 15 or 20");
  int K = t->taps;
  if (!(K == 2 || K == 4 || K == 6 || K == 8 || K == 12 || K == 16 || K == 24 || K == 32))
    return fail(LT_ERR_UNSUPPORTED, "taps must be one of 2,4,6,8,12,16,24,32");
  if (t->channels <= 0 || t->channels > 7) return fail(LT_ERR_CONFIG, "channels must be a nonzero subset of A|E|T");
  double HY = 7.0 * (o->arm_m * 1.01 / kC) / g->dt + K / 2 + 3;
  if (HY > kNodeSpacing - 8) return fail(LT_ERR_UNSUPPORTED, "dt too small for the TDI halo");
  return LT_OK;
}

static GridDev gdev(const lt_grid* g) { return GridDev{g->t0, g->dt, 1.0 / g->dt, g->n}; }

static lt_status do_setup(lt_ctx* c, const double* params, int64_t batch, const lt_wf_cfg* cfg, const lt_grid* g,
                          int32_t* status, hipStream_t s) {
  LT_HIP(c->tpl.ensure((size_t)batch * sizeof(TplConst)));
  Prof pr(c, 0, s);
  LT_HIP(launch_setup(params, batch, cfg->f_low, cfg->f_ref, gdev(g), (TplConst*)c->tpl.p, status, s));
  return LT_OK;
}

// ------------------------------------------------------------------ API
extern "C" {

const char* lt_last_error(void) { return g_err.c_str(); }

lt_status lt_ctx_create(int hip_device, lt_ctx** out) {
  if (!out) return fail(LT_ERR_NULL, "null output pointer");
  int n = 0;
  LT_HIP(hipGetDeviceCount(&n));
  if (hip_device < 0 || hip_device >= n) return fail(LT_ERR_CONFIG, "no such HIP device");
  LT_HIP(hipSetDevice(hip_device));
  void* fixed = nullptr;
  LT_HIP(fixed_scratch(hip_device, &fixed));
  lt_ctx* c = new lt_ctx();
  c->device = hip_device;
  c->scratch = fixed;
  *out = c;
  return LT_OK;
}

lt_status lt_ctx_destroy(lt_ctx* c) {
  if (!c) return fail(LT_ERR_NULL, "null context");
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  drain_profile(c);
  delete c;
  return LT_OK;
}

lt_status lt_phenomt_modes(lt_ctx* c, const double* params, int64_t batch, const lt_wf_cfg* cfg, const lt_grid* g,
                           double* modes, void* stream) {
  lt_status st = check_common(c, params, batch, cfg, g);
  if (st) return st;
  if (!modes) return fail(LT_ERR_NULL, "null modes");
  hipStream_t s = (hipStream_t)stream;
  st = do_setup(c, params, batch, cfg, g, nullptr, s);
  if (st) return st;
  Prof pr(c, 0, s);
  LT_HIP(launch_modes((TplConst*)c->tpl.p, batch, cfg->mode_mask, gdev(g), modes, s));
  return LT_OK;
}

lt_status lt_phenomt_polarizations(lt_ctx* c, const double* params, int64_t batch, const lt_wf_cfg* cfg,
                                   const lt_grid* g, double* hpc, void* stream) {
  lt_status st = check_common(c, params, batch, cfg, g);
  if (st) return st;
  if (!hpc) return fail(LT_ERR_NULL, "null output");
  hipStream_t s = (hipStream_t)stream;
  st = do_setup(c, params, batch, cfg, g, nullptr, s);
  if (st) return st;
  Prof pr(c, 0, s);
  LT_HIP(launch_polarizations((TplConst*)c->tpl.p, batch, cfg->mode_mask, cfg->precessing, cfg->coarse, gdev(g), hpc,
                              s));
  return LT_OK;
}

// Response kernels for `batch` templates whose constants tc are set up: waveform into `wave`
// ([batch][2][n] in the precision's real type), the per-launch tables into `nodes` and `refs`
// (sizes from tdi_scratch_bytes), the fused response into `out`.
// refs_ready: refs already hold the term references of this configuration (an earlier chunk of
// the same call computed them)
static lt_status run_tdi_core(lt_ctx* c, const TplConst* tc, int64_t batch, const lt_wf_cfg* cfg, const lt_grid* g,
                              const OrbitDev& od, const lt_tdi_cfg* t, int out_mode, const void* data, void* out,
                              int32_t* status, void* wave, double* nodes, void* refs, hipStream_t s,
                              bool refs_ready = false) {
  {
    Prof pr(c, 5, s);
    LT_HIP(launch_wave(tc, batch, cfg->mode_mask, cfg->precessing, cfg->coarse, cfg->precision, gdev(g), wave, s));
  }
  TdiLaunch L;
  L.tc = tc;
  L.batch = batch;
  L.h = wave;
  L.taps = t->taps;
  L.comb = 1;
  L.precision = cfg->precision;
  L.out_mode = out_mode;
  L.g = gdev(g);
  L.orb = od;
  L.terms = make_terms(t->generation);
  L.data = data;
  L.out = out;
  L.status = status;
  L.rotate = c->tune.rotate;
  L.persistent = c->tune.persistent;
  L.wg_per_cu = c->tune.wg_per_cu;
  L.nodes = nodes;
  L.refs = refs;
  L.refs_ready = refs_ready ? 1 : 0;
  {
    Prof pr(c, 0, s);
    LT_HIP(launch_tdi(L, 0, s));
  }
  Prof pr(c, 1, s);
  LT_HIP(launch_tdi(L, 1, s));
  return LT_OK;
}

// scratch bytes of the per-launch tables for `batch` templates (0 for an unsupported tap count)
static void tdi_table_bytes(int64_t batch, const lt_wf_cfg* cfg, const lt_grid* g, const lt_tdi_cfg* t,
                            size_t* nb, size_t* rb) {
  TdiLaunch L;
  std::memset(&L, 0, sizeof(L));
  L.batch = batch;
  L.taps = t->taps;
  L.precision = cfg->precision;
  L.g = gdev(g);
  L.orb.n_nodes = orbit_node_count(g);
  tdi_scratch_bytes(L, nb, rb);
}

// the response entry point: the whole batch in one launch, scratch owned by the context
static lt_status run_tdi(lt_ctx* c, const double* params, int64_t batch, const lt_wf_cfg* cfg, const lt_grid* g,
                         const lt_orbit* o, const lt_tdi_cfg* t, int out_mode, void* out, int32_t* status,
                         hipStream_t s) {
  OrbitDev od;
  lt_status st = get_orbit(c, o, g, &od);
  if (st) return st;
  st = do_setup(c, params, batch, cfg, g, status, s);
  if (st) return st;
  const size_t rsz = cfg->precision == LT_FP64 ? sizeof(double) : sizeof(float);
  LT_HIP(c->wave.ensure((size_t)batch * 2 * g->n * rsz));
  size_t nb = 0, rb = 0;
  tdi_table_bytes(batch, cfg, g, t, &nb, &rb);
  if (rb == 0) return fail(LT_ERR_UNSUPPORTED, "unsupported tap count");
  LT_HIP(c->nodes.ensure(nb));
  LT_HIP(c->refs.ensure(rb));
  return run_tdi_core(c, (const TplConst*)c->tpl.p, batch, cfg, g, od, t, out_mode, nullptr, out, status, c->wave.p,
                      (double*)c->nodes.p, c->refs.p, s);
}

lt_status lt_lisa_tdi_response(lt_ctx* c, const double* params, int64_t batch, const lt_wf_cfg* cfg, const lt_grid* g,
                               const lt_orbit* o, const lt_tdi_cfg* t, void* out, int32_t* status, void* stream) {
  lt_status st = check_common(c, params, batch, cfg, g);
  if (st) return st;
  st = check_tdi(o, t, g);
  if (st) return st;
  if (!out) return fail(LT_ERR_NULL, "null output");
  return run_tdi(c, params, batch, cfg, g, o, t, t->out_xyz ? 1 : 0, out, status, (hipStream_t)stream);
}

static lt_status band_bins(const lt_grid* g, const lt_psd* psd, int* k_lo, int* k_hi) {
  const double T = (double)g->n * g->dt;
  const double slack = 1e-12;
  int64_t lo = (int64_t)std::ceil(psd->f_lo * T * (1.0 - slack));
  int64_t hi = (int64_t)std::floor(psd->f_hi * T * (1.0 + slack));
  if (lo < 0) lo = 0;
  if (hi > g->n / 2) hi = g->n / 2;
  if (!(psd->f_hi > psd->f_lo) || hi < lo) return fail(LT_ERR_CONFIG, "empty likelihood band");
  *k_lo = (int)lo;
  *k_hi = (int)hi;
  return LT_OK;
}

// FFT both passes over rows of [rows][n] (in place), band power into `partial`
// (band weights in wperm)
static lt_status fft_band(lt_ctx* c, Plan* p, void* series, int64_t rows, int precision, int k_lo, int k_hi,
                          const lt_grid* g, double* partial, const double* wperm, const int32_t* skip,
                          hipStream_t s) {
  {
    Prof pr(c, 2, s);
    LT_HIP(launch_fft_pass1(p->dev, series, rows, precision, skip, s));
  }
  Prof pr(c, 3, s);
  LT_HIP(launch_fft_pass2(p->dev, series, rows, precision, 1, g->dt, nullptr, wperm, 3, partial, k_lo, k_hi, skip,
                          s));
  return LT_OK;
}

// FFT both passes over rows of [rows][n] (in place), band power into partials
static lt_status band_power(lt_ctx* c, Plan* p, void* series, int64_t rows, int precision, const lt_psd* psd,
                            const lt_grid* g, int channels, hipStream_t s) {
  int k_lo, k_hi;
  lt_status st = band_bins(g, psd, &k_lo, &k_hi);
  if (st) return st;
  const int64_t n = p->dev.n;
  LT_HIP(c->wperm.ensure((size_t)3 * (n + 1) * sizeof(double)));
  LT_HIP(c->partial.ensure((size_t)rows * (p->dev.n1 / 2 + 1) * sizeof(double)));
  {
    Prof pr(c, 0, s);   // per-call table, timed with the setup
    LT_HIP(launch_weights(p->dev, psd->S, k_lo, k_hi, channels, (double*)c->wperm.p, s));
  }
  {
    Prof pr(c, 2, s);
    LT_HIP(launch_fft_pass1(p->dev, series, rows, precision, nullptr, s));
  }
  {
    Prof pr(c, 3, s);
    LT_HIP(launch_fft_pass2(p->dev, series, rows, precision, 1, g->dt, nullptr, (const double*)c->wperm.p, 3,
                            (double*)c->partial.p, k_lo, k_hi, nullptr, s));
  }
  return LT_OK;
}

// ------------------------------------------------------------ likelihood scratch
// One block of device memory per lt_tdi_loglike call, carved into the arrays one chunk of
// templates needs; each array starts on a 256-byte boundary.
struct LoglikeScratch {
  TplConst* tpl;      // [batch] template constants (set up for the whole call in one launch)
  int32_t* status;    // [batch] when the caller passes no status array
  double* wperm;      // [3][n + 1] band weights in pass-2 order
  void* work;         // [chunk][3][n] residual, transformed in place
  double* partial;    // [chunk][3][n1/2 + 1] band partial sums
  void* wave;         // [chunk][2][n] polarisations
  double* nodes;      // per-launch node records and window bounds
  void* refs;         // per-launch term references and combined filters
};

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// bytes of the scratch of a call over `batch` templates in chunks of `chunk`, and (base != null)
// the arrays within it
static size_t loglike_layout(int64_t chunk, int64_t batch, const lt_wf_cfg* cfg, const lt_grid* g,
                             const lt_tdi_cfg* t, int nfold, unsigned char* base, LoglikeScratch* out) {
  const size_t rsz = cfg->precision == LT_FP64 ? sizeof(double) : sizeof(float);
  size_t nb = 0, rb = 0;
  tdi_table_bytes(chunk, cfg, g, t, &nb, &rb);
  const size_t parts[8] = {(size_t)batch * sizeof(TplConst), (size_t)batch * sizeof(int32_t),
                           (size_t)3 * (g->n + 1) * sizeof(double), (size_t)chunk * 3 * g->n * rsz,
                           (size_t)chunk * 3 * nfold * sizeof(double), (size_t)chunk * 2 * g->n * rsz, nb, rb};
  size_t off[8], total = 0;
  for (int i = 0; i < 8; ++i) {
    off[i] = total;
    total += align256(parts[i]);
  }
  if (base && out) {
    out->tpl = (TplConst*)(base + off[0]);
    out->status = (int32_t*)(base + off[1]);
    out->wperm = (double*)(base + off[2]);
    out->work = base + off[3];
    out->partial = (double*)(base + off[4]);
    out->wave = base + off[5];
    out->nodes = (double*)(base + off[6]);
    out->refs = base + off[7];
  }
  return total;
}

// largest chunk (at most `cap` and the batch) whose scratch fits `bytes`; 0 if none does
static int64_t loglike_chunk_for(size_t bytes, int64_t batch, const lt_wf_cfg* cfg, const lt_grid* g,
                                 const lt_tdi_cfg* t, int nfold, int64_t cap) {
  int64_t hi = batch < cap ? batch : cap;
  if (loglike_layout(hi, batch, cfg, g, t, nfold, nullptr, nullptr) <= bytes) return hi;
  int64_t lo = 0;   // invariant: layout(lo) fits (or lo = 0), layout(hi) does not
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) / 2;
    if (loglike_layout(mid, batch, cfg, g, t, nfold, nullptr, nullptr) <= bytes) lo = mid;
    else hi = mid;
  }
  return lo;
}

static lt_status check_loglike(lt_ctx* c, const double* params, int64_t batch, const lt_wf_cfg* cfg,
                               const lt_grid* g, const lt_orbit* o, const lt_tdi_cfg* t, const lt_psd* psd,
                               const lt_data* data, const double* logl, const double* logl_full, int* nfold) {
  lt_status st = check_common(c, params, batch, cfg, g);
  if (st) return st;
  st = check_tdi(o, t, g);
  if (st) return st;
  if (!psd || !psd->S[0] || !psd->S[1] || !psd->S[2]) return fail(LT_ERR_NULL, "null PSD");
  if (!data || !data->aet) return fail(LT_ERR_NULL, "null data");
  if (!logl && !logl_full) return fail(LT_ERR_NULL, "no output requested");
  int n1, n2;
  if (!plan_shape(g->n, &n1, &n2))
    return fail(LT_ERR_UNSUPPORTED, "N/2 must factor as n1*n2 (n1 even, both <= 1024) over radices 2,3,5");
  *nfold = n1 / 2 + 1;
  size_t nb = 0, rb = 0;
  tdi_table_bytes(1, cfg, g, t, &nb, &rb);
  if (rb == 0) return fail(LT_ERR_UNSUPPORTED, "unsupported tap count");
  return LT_OK;
}

// The likelihood over `batch` templates in chunks of `chunk`, with all per-call memory in `base`
// (laid out by loglike_layout for that chunk).  may_alloc false: the FFT plan and the orbit
// table must already be in the context.
static lt_status loglike_run(lt_ctx* c, const double* params, int64_t batch, const lt_wf_cfg* cfg, const lt_grid* g,
                             const lt_orbit* o, const lt_tdi_cfg* t, const lt_psd* psd, const lt_data* data,
                             double* logl, double* logl_full, int32_t* status, int nfold, int64_t chunk,
                             unsigned char* base, bool may_alloc, hipStream_t s) {
  Plan* p;
  lt_status st = get_plan(c, g->n, &p, may_alloc);
  if (st) return st;
  OrbitDev od;
  st = get_orbit(c, o, g, &od, may_alloc);
  if (st) return st;
  int k_lo, k_hi;
  st = band_bins(g, psd, &k_lo, &k_hi);
  if (st) return st;
  LoglikeScratch w;
  loglike_layout(chunk, batch, cfg, g, t, nfold, base, &w);
  const double scale = 4.0 * g->dt / (double)g->n;
  int32_t* stat_all = status ? status : w.status;
  {
    Prof pr(c, 0, s);   // per-call table and set-up
    LT_HIP(launch_weights(p->dev, psd->S, k_lo, k_hi, t->channels, w.wperm, s));
    // every template's constants in one launch: a thread's set-up is a long serial FP64 chain,
    // so one launch per chunk would pay that latency once per chunk
    LT_HIP(launch_setup(params, batch, cfg->f_low, cfg->f_ref, gdev(g), w.tpl, stat_all, s));
  }
  // one stream, chunks of templates: the response kernel already fills the GPU, and running a
  // chunk's FFT beside the next chunk's response on a second stream measured no faster than this
  for (int64_t off = 0; off < batch; off += chunk) {
    const int64_t b = batch - off < chunk ? batch - off : chunk;
    int32_t* stat = stat_all + off;
    st = run_tdi_core(c, w.tpl + off, b, cfg, g, od, t, 2, data->aet, w.work, stat, w.wave, w.nodes, w.refs, s,
                      off > 0);
    if (st) return st;
    st = fft_band(c, p, w.work, b * 3, cfg->precision, k_lo, k_hi, g, w.partial, w.wperm, stat, s);
    if (st) return st;
    Prof pr(c, 4, s);
    LT_HIP(launch_finalize(w.partial, b, nfold, scale, data->dd, stat, logl ? logl + off : nullptr,
                           logl_full ? logl_full + off : nullptr, nullptr, s));
  }
  return LT_OK;
}

lt_status lt_workspace_size(lt_ctx* c, int64_t batch, const lt_wf_cfg* cfg, const lt_grid* g, const lt_tdi_cfg* t,
                            size_t* bytes, size_t* min_bytes) {
  if (!c || !cfg || !g || !t || (!bytes && !min_bytes)) return fail(LT_ERR_NULL, "null argument");
  if (batch < 1 || batch > 65535) return fail(LT_ERR_SHAPE, "batch must be in [1, 65535]");
  if (g->n < 8 || g->n > ((int64_t)1 << 26)) return fail(LT_ERR_SHAPE, "grid n must be in [8, 2^26]");
  if (cfg->precision != LT_FP64 && cfg->precision != LT_MIXED) return fail(LT_ERR_CONFIG, "bad precision");
  int n1, n2;
  if (!plan_shape(g->n, &n1, &n2))
    return fail(LT_ERR_UNSUPPORTED, "N/2 must factor as n1*n2 (n1 even, both <= 1024) over radices 2,3,5");
  size_t nb = 0, rb = 0;
  tdi_table_bytes(1, cfg, g, t, &nb, &rb);
  if (rb == 0) return fail(LT_ERR_UNSUPPORTED, "taps must be one of 2,4,6,8,12,16,24,32");
  const int64_t full = batch < c->tune.chunk ? batch : c->tune.chunk;
  if (bytes) *bytes = loglike_layout(full, batch, cfg, g, t, n1 / 2 + 1, nullptr, nullptr);
  if (min_bytes) *min_bytes = loglike_layout(1, batch, cfg, g, t, n1 / 2 + 1, nullptr, nullptr);
  return LT_OK;
}

lt_status lt_tdi_loglike(lt_ctx* c, const double* params, int64_t batch, const lt_wf_cfg* cfg, const lt_grid* g,
                         const lt_orbit* o, const lt_tdi_cfg* t, const lt_psd* psd, const lt_data* data, double* logl,
                         double* logl_full, int32_t* status, void* workspace, size_t workspace_bytes, void* stream) {
  int nfold;
  lt_status st = check_loglike(c, params, batch, cfg, g, o, t, psd, data, logl, logl_full, &nfold);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  int64_t chunk;
  unsigned char* base;
  if (workspace) {
    chunk = loglike_chunk_for(workspace_bytes, batch, cfg, g, t, nfold, c->tune.chunk);
    if (chunk < 1) return fail(LT_ERR_WORKSPACE, "workspace smaller than one template needs (lt_workspace_size)");
    base = (unsigned char*)workspace;
  } else {
    chunk = batch < c->tune.chunk ? batch : c->tune.chunk;
    LT_HIP(c->ws.ensure(loglike_layout(chunk, batch, cfg, g, t, nfold, nullptr, nullptr)));
    base = (unsigned char*)c->ws.p;
  }
  return loglike_run(c, params, batch, cfg, g, o, t, psd, data, logl, logl_full, status, nfold, chunk, base, true, s);
}

lt_status lt_tdi_loglike_noalloc(lt_ctx* c, const double* params, int64_t batch, const lt_wf_cfg* cfg,
                                 const lt_grid* g, const lt_orbit* o, const lt_tdi_cfg* t, const lt_psd* psd,
                                 const lt_data* data, double* logl, double* logl_full, int32_t* status,
                                 void* stream) {
  int nfold;
  lt_status st = check_loglike(c, params, batch, cfg, g, o, t, psd, data, logl, logl_full, &nfold);
  if (st) return st;
  if (!c->scratch) return fail(LT_ERR_DEVICE, "no fixed scratch on this device");
  const int64_t chunk = loglike_chunk_for(kFixedScratchBytes, batch, cfg, g, t, nfold, c->tune.chunk);
  if (chunk < 1) {
    const size_t need = loglike_layout(1, batch, cfg, g, t, nfold, nullptr, nullptr);
    return fail(LT_ERR_WORKSPACE, "chunks of one template of this batch and grid need " + std::to_string(need) +
                                      " bytes of scratch, more than the fixed " +
                                      std::to_string(kFixedScratchBytes) + " (use lt_tdi_loglike)");
  }
  // no profiling events either: this path creates nothing
  const bool prof = c->profiling;
  c->profiling = false;
  st = loglike_run(c, params, batch, cfg, g, o, t, psd, data, logl, logl_full, status, nfold, chunk,
                   (unsigned char*)c->scratch, false, (hipStream_t)stream);
  c->profiling = prof;
  return st;
}

lt_status lt_ctx_set_tuning(lt_ctx* c, const lt_tuning* t) {
  if (!c) return fail(LT_ERR_NULL, "null context");
  if (!t) {
    c->tune = lt_tuning{256, 1, 0, 4};
    return LT_OK;
  }
  if (t->chunk < 1 || t->chunk > 4096) return fail(LT_ERR_CONFIG, "chunk must be in [1, 4096]");
  if ((t->rotate != 0 && t->rotate != 1) || (t->persistent != 0 && t->persistent != 1))
    return fail(LT_ERR_CONFIG, "rotate and persistent must be 0 or 1");
  if (t->wg_per_cu < 1 || t->wg_per_cu > 16) return fail(LT_ERR_CONFIG, "wg_per_cu must be in [1, 16]");
  c->tune = *t;
  return LT_OK;
}

lt_status lt_ctx_get_tuning(lt_ctx* c, lt_tuning* t) {
  if (!c || !t) return fail(LT_ERR_NULL, "null argument");
  *t = c->tune;
  return LT_OK;
}

// the workload key of a cached tuning
static std::string tune_key(lt_ctx* c, int64_t batch, const lt_wf_cfg* cfg, const lt_grid* g, const lt_tdi_cfg* t) {
  hipDeviceProp_t prop;
  std::ostringstream k;
  if (hipGetDeviceProperties(&prop, c->device) == hipSuccess)
    k << prop.gcnArchName << ":" << prop.multiProcessorCount << "cu";
  else
    k << "unknown";
  k << "|n=" << g->n << "|prec=" << cfg->precision << "|taps=" << t->taps << "|gen=" << t->generation
    << "|modes=" << cfg->mode_mask << "|prec_spin=" << cfg->precessing << "|coarse=" << cfg->coarse
    << "|batch=" << batch;
  std::string s = k.str();
  for (char& ch : s)
    if (ch == ' ' || ch == '\t') ch = '_';
  return s;
}

lt_status lt_autotune(lt_ctx* c, const double* params, int64_t batch, const lt_wf_cfg* cfg, const lt_grid* g,
                      const lt_orbit* o, const lt_tdi_cfg* t, const lt_psd* psd, const lt_data* data,
                      const char* cache_path, int reps, lt_tuning* best, double* best_ms, void* stream) {
  int nfold;
  double unused = 0.0;   // the outputs are the tuner's own
  lt_status st = check_loglike(c, params, batch, cfg, g, o, t, psd, data, &unused, nullptr, &nfold);
  if (st) return st;
  if (reps < 1 || reps > 1000) return fail(LT_ERR_CONFIG, "reps must be in [1, 1000]");
  const std::string key = tune_key(c, batch, cfg, g, t);
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    lt_tuning found{0, 0, 0, 0};
    bool have = false;
    while (std::getline(in, line)) {
      std::istringstream ls(line);
      std::string k;
      lt_tuning v{0, 0, 0, 0};
      if (ls >> k >> v.chunk >> v.rotate >> v.persistent >> v.wg_per_cu && k == key) {
        found = v;
        have = true;      // the last entry for the key wins
      }
    }
    if (have && lt_ctx_set_tuning(c, &found) == LT_OK) {
      if (best) *best = found;
      if (best_ms) *best_ms = -1.0;
      return LT_OK;
    }
  }
  hipStream_t s = (hipStream_t)stream;
  std::vector<lt_tuning> cand;
  for (int chunk : {256, 64, 128, 512}) {
    if (chunk > 256 && chunk / 2 >= batch) continue;   // no larger chunk than the batch needs
    if (chunk < 256 && chunk >= batch) continue;
    for (int rot : {1, 0}) {
      cand.push_back({chunk, rot, 0, 4});
      cand.push_back({chunk, rot, 1, 4});
      cand.push_back({chunk, rot, 1, 8});
    }
  }
  LT_HIP(c->tune_out.ensure((size_t)batch * sizeof(double)));
  double* out = (double*)c->tune_out.p;
  std::vector<double> ref((size_t)batch), got((size_t)batch);
  hipEvent_t e0, e1;
  LT_HIP(hipEventCreate(&e0));
  LT_HIP(hipEventCreate(&e1));
  const lt_tuning saved = c->tune;
  c->tune_discarded = 0;
  double bms = 1e300;
  lt_tuning bt = saved;
  // every candidate once (warm-up, sizes its scratch, checks its results against the default
  // shape's), then three rounds of `reps` timed calls each, candidates interleaved so that a
  // drift of the clocks hits all of them; a candidate's time is its best round
  std::vector<double> tbest(cand.size(), 1e300);
  for (int round = -1; round < 3 && st == LT_OK; ++round) {
    for (size_t i = 0; i < cand.size() && st == LT_OK; ++i) {
      c->tune = cand[i];
      const int calls = round < 0 ? 1 : reps;
      if (hipEventRecord(e0, s) != hipSuccess) { st = fail(LT_ERR_DEVICE, "event record"); break; }
      for (int r = 0; r < calls && st == LT_OK; ++r)
        st = lt_tdi_loglike(c, params, batch, cfg, g, o, t, psd, data, out, nullptr, nullptr, nullptr, 0, stream);
      if (st) break;
      float ms = 0.f;
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        st = fail(LT_ERR_DEVICE, "autotune timing");
        break;
      }
      if (round < 0) {
        if (hipMemcpy(got.data(), out, (size_t)batch * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
          st = fail(LT_ERR_DEVICE, "autotune copy");
          break;
        }
        if (i == 0) ref = got;
        if (std::memcmp(ref.data(), got.data(), ref.size() * sizeof(double)) != 0) ++c->tune_discarded;
      } else {
        tbest[i] = std::min(tbest[i], (double)ms / reps);
      }
    }
  }
  for (size_t i = 0; i < cand.size(); ++i)
    if (tbest[i] < bms) {
      bms = tbest[i];
      bt = cand[i];
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) {
    c->tune = saved;
    return st;
  }
  c->tune = bt;
  if (c->tune_discarded) return fail(LT_ERR_DEVICE, "autotune: a launch shape changed the results");
  if (best) *best = bt;
  if (best_ms) *best_ms = bms;
  if (cache_path) {
    std::ofstream outf(cache_path, std::ios::app);
    if (outf) outf << key << " " << bt.chunk << " " << bt.rotate << " " << bt.persistent << " " << bt.wg_per_cu << " "
                   << bms << "\n";
  }
  return LT_OK;
}

lt_status lt_noise_inner(lt_ctx* c, const void* x, int64_t batch, const lt_grid* g, const lt_psd* psd, int channels,
                         int precision, double* out, void* stream) {
  if (!c) return fail(LT_ERR_NULL, "null context");
  if (!x || !g || !psd || !out || !psd->S[0] || !psd->S[1] || !psd->S[2]) return fail(LT_ERR_NULL, "null argument");
  if (batch < 1 || batch > 65535) return fail(LT_ERR_SHAPE, "batch must be in [1, 65535]");
  if (precision != LT_FP64 && precision != LT_MIXED) return fail(LT_ERR_CONFIG, "bad precision");
  if (channels <= 0 || channels > 7) return fail(LT_ERR_CONFIG, "bad channels");
  LT_HIP(hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  Plan* p;
  lt_status st = get_plan(c, g->n, &p);
  if (st) return st;
  const size_t rsz = precision == LT_FP64 ? sizeof(double) : sizeof(float);
  const size_t bytes = (size_t)batch * 3 * g->n * rsz;
  LT_HIP(c->work.ensure(bytes));
  LT_HIP(hipMemcpyAsync(c->work.p, x, bytes, hipMemcpyDeviceToDevice, s));
  st = band_power(c, p, c->work.p, batch * 3, precision, psd, g, channels, s);
  if (st) return st;
  Prof pr(c, 4, s);
  LT_HIP(launch_finalize((const double*)c->partial.p, batch, p->dev.n1 / 2 + 1, 4.0 * g->dt / (double)g->n, 0.0,
                         nullptr, nullptr, nullptr, out, s));
  return LT_OK;
}

lt_status lt_rfft(lt_ctx* c, const void* x, int64_t rows, int64_t n, double dt, int precision, void* spec,
                  void* stream) {
  if (!c) return fail(LT_ERR_NULL, "null context");
  if (!x || !spec) return fail(LT_ERR_NULL, "null argument");
  if (rows < 1 || rows > 65535) return fail(LT_ERR_SHAPE, "rows must be in [1, 65535]");
  if (precision != LT_FP64 && precision != LT_MIXED) return fail(LT_ERR_CONFIG, "bad precision");
  LT_HIP(hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  Plan* p;
  lt_status st = get_plan(c, n, &p);
  if (st) return st;
  const size_t rsz = precision == LT_FP64 ? sizeof(double) : sizeof(float);
  const size_t bytes = (size_t)rows * n * rsz;
  LT_HIP(c->work.ensure(bytes));
  LT_HIP(hipMemcpyAsync(c->work.p, x, bytes, hipMemcpyDeviceToDevice, s));
  {
    Prof pr(c, 2, s);
    LT_HIP(launch_fft_pass1(p->dev, c->work.p, rows, precision, nullptr, s));
  }
  Prof pr(c, 3, s);
  LT_HIP(launch_fft_pass2(p->dev, c->work.p, rows, precision, 0, dt, spec, nullptr, 3, nullptr, 0, p->dev.n, nullptr,
                          s));
  return LT_OK;
}

lt_status lt_psd_sangria(const lt_grid* g, int generation, double arm_m, double* S, void* stream) {
  if (!g || !S) return fail(LT_ERR_NULL, "null argument");
  if (g->n < 8 || !(g->dt > 0.0)) return fail(LT_ERR_SHAPE, "bad grid");
  if (generation != 15 && generation != 20) return fail(LT_ERR_CONFIG, "generation must be 15 or 20");
  const int64_t nb = g->n / 2 + 1;
  std::vector<double> h(3 * nb);
  for (int64_t k = 0; k < nb; ++k) {
    if (k == 0) {
      h[k] = h[nb + k] = h[2 * nb + k] = INFINITY;
      continue;
    }
    double f = (double)k / ((double)g->n * g->dt);
    double x = 2.0 * M_PI * f * arm_m / kC;
    double w = 2.0 * M_PI * f / kC;
    double sacc = 2.4e-15 * 2.4e-15 * (1.0 + std::pow(4e-4 / f, 2)) * (1.0 + std::pow(f / 8e-3, 4)) *
                  std::pow(2.0 * M_PI * f, -4) * w * w;
    double sop = 7.9e-12 * 7.9e-12 * (1.0 + std::pow(2e-3 / f, 4)) * w * w;
    double s2 = std::sin(x) * std::sin(x);
    double ae = 8.0 * s2 * (2.0 * sacc * (3.0 + 2.0 * std::cos(x) + std::cos(2.0 * x)) + sop * (2.0 + std::cos(x)));
    double tt = 16.0 * sop * (1.0 - std::cos(x)) * s2 + 128.0 * sacc * s2 * std::pow(std::sin(0.5 * x), 4);
    if (generation == 20) {
      double f2 = 4.0 * std::sin(2.0 * x) * std::sin(2.0 * x);
      ae *= f2;
      tt *= f2;
    }
    h[k] = ae;
    h[nb + k] = ae;
    h[2 * nb + k] = tt;
  }
  LT_HIP(hipMemcpyAsync(S, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, (hipStream_t)stream));
  LT_HIP(hipStreamSynchronize((hipStream_t)stream));
  return LT_OK;
}

lt_status lt_profile_enable(lt_ctx* c, int on) {
  if (!c) return fail(LT_ERR_NULL, "null context");
  c->profiling = on != 0;
  return LT_OK;
}

lt_status lt_profile_read(lt_ctx* c, double* ms, int64_t* launches, int n_classes) {
  if (!c || !ms || !launches) return fail(LT_ERR_NULL, "null argument");
  drain_profile(c);
  for (int i = 0; i < n_classes && i < 8; ++i) {
    ms[i] = c->prof_ms[i];
    launches[i] = c->prof_n[i];
    c->prof_ms[i] = 0.0;
    c->prof_n[i] = 0;
  }
  return LT_OK;
}

}  // extern "C"
