// Launch interfaces of the liblisatd kernels (host side).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "lt_common.hpp"

namespace lt {

// One TDI term: sign * y_link(t - sum_k dcnt[k] L_{dlink[k]}(t)); links
// indexed 0..5 for the labels 1, 2, 3, -1, -2, -3.
struct Term { int sign, link, nd, dlink[4], dcnt[4]; };
// Terms of one channel that read the same link form a group (at most 4 links
// and 8 terms per group); max_delays bounds the number of light times summed
// in one term delay.
struct TermTable {
  int n_terms[3];
  Term t[3][16];
  int n_groups[3], g_link[3][4], g_n[3][4], g_t[3][4][8];
  int max_delays;
  double g_span;      // max over groups of (max - min) light times summed, + 5 % of the min (arm flexing)
};

// Orbit node table on the device: node j sits at grid sample (j - j0) * spacing;
// per node and link: L [s], r_receiver / c [s] (3), r_sender(emission) / c [s] (3), n (3).
constexpr int kNodeLink = 10;
constexpr int kNodeStride = 6 * kNodeLink;
struct OrbitDev {
  const double* tab;
  int n_nodes, j0, spacing;
  double max_light_time;
};

struct GridDev { double t0, dt, inv_dt; int64_t n; };

hipError_t launch_setup(const double* params, int64_t batch, double f_low, double f_ref, GridDev g,
                        TplConst* tc, int32_t* status, hipStream_t s);
hipError_t launch_modes(const TplConst* tc, int64_t batch, int mode_mask, GridDev g, double* modes,
                        hipStream_t s);
// coarse 2: waveform on the even samples, odd samples the mean of their neighbours
hipError_t launch_polarizations(const TplConst* tc, int64_t batch, int mode_mask, int precessing, int coarse,
                                GridDev g, double* hpc, hipStream_t s);
// h: [batch][2][n], double (precision 0) or float (precision 1)
hipError_t launch_wave(const TplConst* tc, int64_t batch, int mode_mask, int precessing, int coarse, int precision,
                       GridDev g, void* h, hipStream_t s);

// out_mode: 0 write A,E,T; 1 write X,Y,Z; 2 write A,E,T minus data (residual)
struct TdiLaunch {
  const TplConst* tc;
  int64_t batch;
  int taps, precision, out_mode;
  int comb;           // mixed precision: per-link combined filters (phase D) allowed
  GridDev g;
  OrbitDev orb;
  TermTable terms;
  const void* h;      // waveform buffer [batch][2][n]
  const void* data;   // [3][n] (residual mode)
  void* out;          // [batch][3][n]
  int32_t* status;    // nullable
  double* nodes;      // scratch: response geometry per (template, orbit node), then the window bounds
  void* refs;         // scratch: TDI term references and combined filters per tile
  int* win;           // set by launch_tdi: window bounds per (template, tile), after the node records
  // launch shape (results do not depend on it): rotate the template order with the tile; one
  // persistent grid of wg_per_cu workgroups per CU taking (template, tile) items from a counter
  // instead of one workgroup per item
  int rotate = 1;
  int persistent = 0;
  int wg_per_cu = 4;
  unsigned long long* counter;   // set by launch_tdi: the persistent grid's item counter, after the records
  // 1: refs already hold this configuration's term references and filters (they depend on the
  // grid, orbit and TDI configuration, not on the templates): the tables stage skips them
  int refs_ready = 0;
};
// stage 0: the per-launch tables (node geometry, term references, combined filters);
// stage 1: the response kernel itself
hipError_t launch_tdi(const TdiLaunch& L, int stage, hipStream_t s);
// scratch bytes of launch_tdi for L (L.batch, taps, precision, grid and orbit set)
void tdi_scratch_bytes(const TdiLaunch& L, size_t* nodes, size_t* refs);
int tdi_tile();

// ---------------------------------------------------------------- FFT
struct FftPlanDev {
  int64_t N, n;          // real length, complex length n = N/2
  int n1, n2;            // n = n1 * n2 (pass 1: FFTs of length n1 over columns, pass 2: length n2 rows)
  int rad1[12], nr1, rad2[12], nr2;
  const double* tw1d; const float* tw1f;    // exp(-2 pi i k / n1), k < n1 (complex interleaved)
  const double* tw2d; const float* tw2f;    // exp(-2 pi i k / n2)
  const double* wlod; const float* wlof;    // exp(-2 pi i k / N), k < 1024
  const double* whid; const float* whif;    // exp(-2 pi i 1024 k / N), k <= N/1024
};

// skip (nullable): per-template status; rows 3b .. 3b + 2 of a template with nonzero status are
// not transformed (pass 2 writes no partial sums for them)
hipError_t launch_fft_pass1(const FftPlanDev& p, void* data, int64_t rows, int precision, const int32_t* skip,
                            hipStream_t s);
// mode 0: spectrum out[row][k] = R_k * dt (k = 0..n); mode 1: band power partial sums
// mode 1 (band power) reads weights and accumulates only for bins kb_lo..kb_hi
hipError_t launch_fft_pass2(const FftPlanDev& p, const void* data, int64_t rows, int precision, int mode,
                            double dt, void* spec_out, const double* wperm, int64_t ch_stride_rows,
                            double* partial, int64_t kb_lo, int64_t kb_hi, const int32_t* skip, hipStream_t s);
hipError_t launch_weights(const FftPlanDev& p, const double* const* S, int k_lo, int k_hi, int channels,
                          double* wperm, hipStream_t s);
// out[b] = scale * sum_{c, pairs} partial; logl variant adds dd/2 and handles status
hipError_t launch_finalize(const double* partial, int64_t batch, int npairs, double scale, double dd,
                           int32_t* status, double* logl, double* logl_full, double* inner,
                           hipStream_t s);

}  // namespace lt
