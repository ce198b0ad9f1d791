/*
 * liblisatd -- MI355X (gfx950) time-domain LISA likelihood.
 *
 * C ABI of the hot path of arXiv:2501.08261 ("GPU-accelerated LISA parameter
 * estimation with full time domain response"): per template, IMRPhenomT-form
 * modes (Sec. II.A) twisted up through Euler angles and quaternions
 * (Eqs. 2.4-2.6), projected on the six LISA links (Eq. 2.8), combined into
 * TDI 1.5 / 2.0 X, Y, Z (Eqs. 2.9-2.10) and A, E, T (Eq. 2.11), Fourier
 * transformed and reduced to the PSD-weighted log-likelihood
 * (Eqs. 2.12-2.13, with the PSD of Eqs. 2.14-2.15).
 *
 * Conventions shared by every entry point:
 *  - Every call returns lt_status (0 on success, < 0 on error) and never
 *    throws or aborts.  lt_last_error() returns a thread-local message for
 *    the last failing call.
 *  - "device" pointers are HIP device memory owned by the caller; the library
 *    never frees caller memory.  Calls are asynchronous and ordered on the
 *    given stream (0 = the null stream); outputs are valid once the stream
 *    has been synchronised.  A context may be used by one host thread at a
 *    time.
 *  - Layouts are row-major.  params is FP64 [batch][16]:
 *      0 m1, 1 m2 [solar masses, detector frame]
 *      2-4 chi1 (x, y, z), 5-7 chi2 (x, y, z)  [dimensionless, L0 frame at f_ref]
 *      8 D_L [Mpc], 9 iota, 10 phi_ref, 11 t_c [SSB time of the (2,2) peak, s],
 *      12 lambda (ecliptic longitude), 13 beta (ecliptic latitude), 14 psi, 15 unused
 *    (angles in radians).  Aligned-spin models use chi1z, chi2z only.
 *  - Time series are [batch][3][n]; spectra [rows][n/2+1] complex interleaved.
 *  - Host-checkable faults (null pointers, bad sizes, unsupported options)
 *    return an error synchronously and launch nothing.  Domain faults of a
 *    template are reported per template in `status` (1 = unphysical
 *    parameters, 2 = non-finite result, 3 = delay window overflow; see
 *    lt_tdi_loglike) and give logL = -inf.
 */
#ifndef LISATD_H
#define LISATD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LT_OK = 0,
  LT_ERR_NULL = -1,        /* a required pointer is null */
  LT_ERR_SHAPE = -2,       /* batch / n / sizes out of range */
  LT_ERR_CONFIG = -3,      /* inconsistent option values */
  LT_ERR_UNSUPPORTED = -4, /* option outside what the library implements */
  LT_ERR_DEVICE = -5,      /* HIP runtime or launch failure */
  LT_ERR_WORKSPACE = -6    /* caller workspace too small */
} lt_status;

typedef struct lt_ctx lt_ctx;   /* opaque: FFT plans, twiddles, orbit tables, scratch */

enum { LT_FP64 = 0, LT_MIXED = 1 };                         /* lt_wf_cfg.precision */
enum { LT_ORBIT_STATIC_EQUAL = 0, LT_ORBIT_KEPLER = 1, LT_ORBIT_TABLE = 2 };   /* lt_orbit.kind */
enum { LT_CH_A = 1, LT_CH_E = 2, LT_CH_T = 4 };             /* lt_tdi_cfg.channels */
enum { LT_MODE_22 = 1, LT_MODE_21 = 2, LT_MODE_33 = 4, LT_MODE_32 = 8, LT_MODE_44 = 16 };

/* Uniform SSB time grid t_k = t0 + k dt, k = 0..n-1 (Sec. II.C: dt = 5 s). */
typedef struct { double t0, dt; int64_t n; } lt_grid;

/* Waveform options (Sec. II.A).  mode_mask: OR of LT_MODE_* (co-precessing
 * modes with m > 0; m < 0 follow by symmetry).  precessing: 0 = aligned spins
 * (IMRPhenomT / THM form), 1 = twisted-up precessing (TP / TPHM form).
 * f_low: hard start of the (2,2) mode [Hz]; f_ref: reference frequency of the
 * orbital phase and spins [Hz].  precision: LT_FP64 or LT_MIXED (phase and
 * time FP64; stored polarisations, response, FFT FP32; reductions FP64).
 * coarse: 0 or 1 evaluates the polarisations on every grid sample; 2 evaluates
 * them on every second sample (even indices, a grid of step 2 dt) and takes
 * the mean of the two neighbours on the others (the paper's 10 s waveform grid
 * linearly upsampled to 5 s, Sec. II.C): half the waveform work, at a relative
 * error up to (2 pi f dt)^2 / 2 at frequency f.  Affects the polarisations,
 * the response and the likelihood, not lt_phenomt_modes. */
typedef struct { int mode_mask; int precessing; double f_low, f_ref; int precision; int coarse; } lt_wf_cfg;

/* Spacecraft orbits (Sec. II.B).  STATIC_EQUAL: rigid equilateral triangle of
 * side arm_m centred at (au_m, 0, 0), plane inclined 60 deg; KEPLER: three
 * exact Keplerian ellipses (semi-major axis au_m, eccentricity
 * arm_m / (2 sqrt(3) au_m), inclination sqrt(3) times that), mean anomalies
 * offset by 2 pi/3, guiding centre at longitude phase0 at time t_ref.
 * TABLE: positions and light travel times sampled on a uniform time grid, as
 * orbit files give them (the paper's unequal-arm runs read ESA files, Sec. II.B):
 * pos [n_tab][3][3] (spacecraft 1..3, SSB x, y, z in m) and ltt [n_tab][6]
 * (links 1, 2, 3, -1, -2, -3, light time in s for reception at that time) at
 * times tab_t0 + j tab_dt, host memory.  Between samples both are interpolated
 * with four-point Lagrange weights (samples j-1 .. j+2 around t); the receiver
 * sits at the reception time t and the sender at t - L(t).  The table must cover
 * the grid, with one sample interval and the longest light time to spare (else
 * LT_ERR_CONFIG), and n_tab >= 4.  arm_m stays the nominal arm (PSD, halo bound;
 * the table's light times must not exceed 1.01 arm_m / c); au_m, phase0, t_ref
 * are unused.  The library reads the arrays during the call and caches the
 * device node table under a hash of their contents; a sampler copies them. */
typedef struct {
  int kind;
  double arm_m, au_m, phase0, t_ref;
  int64_t n_tab;
  double tab_t0, tab_dt;
  const double* pos;
  const double* ltt;
} lt_orbit;

/* TDI options (Sec. II.B): generation 15 (Eq. 2.9) or 20 (Eq. 2.10);
 * channels: OR of LT_CH_* used by the likelihood; taps: even Lagrange
 * interpolation order K in {2, 4, 6, 8, 12, 16, 24, 32} (K = 2 is the paper's
 * linear interpolation); out_xyz: 1 makes lt_lisa_tdi_response write X, Y, Z
 * instead of A, E, T. */
typedef struct { int generation; int channels; int taps; int out_xyz; } lt_tdi_cfg;

/* One-sided PSD per channel (A, E, T), device FP64 [n/2+1] each, and the
 * likelihood band [f_lo, f_hi] (Sec. II.C: 3e-4 .. 0.02 Hz). */
typedef struct { const double* S[3]; double f_lo, f_hi; } lt_psd;

/* Data (the zero-noise injection of Sec. II.C): device time series [3][n] of
 * A, E, T in the precision's real type (double for LT_FP64, float for
 * LT_MIXED), and dd = sum_c (d_c|d_c) in FP64 (see lt_noise_inner). */
typedef struct { const void* aet; double dd; } lt_data;

const char* lt_last_error(void);
lt_status lt_ctx_create(int hip_device, lt_ctx** out);
lt_status lt_ctx_destroy(lt_ctx* ctx);

/* Launch shape of the likelihood (lt_tdi_loglike and its variants, lt_lisa_tdi_response).
 * None of it changes a result: every variant computes every output with the same operations
 * in the same order, which the GPU tests check bit for bit.
 *  chunk:      templates per launch of lt_tdi_loglike, 1..4096 (256; bounded by the workspace)
 *  rotate:     1 rotates the template order with the tile in the response kernel's work order
 *              (each of the 8 XCDs then sees every template), 0 keeps it (1)
 *  persistent: 1 runs the response kernel as a persistent grid of wg_per_cu workgroups per
 *              compute unit taking (template, tile) items from a counter, 0 as one
 *              workgroup per item (0)
 *  wg_per_cu:  1..16 (4) */
typedef struct { int chunk; int rotate; int persistent; int wg_per_cu; } lt_tuning;
/* tune = null restores the defaults. */
lt_status lt_ctx_set_tuning(lt_ctx* ctx, const lt_tuning* tune);
lt_status lt_ctx_get_tuning(lt_ctx* ctx, lt_tuning* tune);
/* Autotuner of the launch shape for one workload: when cache_path (nullable) names a file
 * holding an entry for this workload's key (device architecture and compute units, grid
 * length, precision, taps, generation, modes, precessing, coarse, batch), that entry is used;
 * otherwise every candidate shape (chunk 64, 128, 256, 512 up to the batch; rotate 0 / 1;
 * one workgroup per item, or persistent with 4 or 8 workgroups per compute unit) runs
 * lt_tdi_loglike on the given templates and data, once to warm up, then in three rounds of
 * `reps` calls under HIP events on `stream` (candidates interleaved; a candidate's time is its
 * best round); a shape whose logL differs in any bit from the default shape's makes
 * the call fail with LT_ERR_DEVICE (a broken invariance, never expected), else the fastest
 * is chosen and appended to the file.  The choice is set on the context and returned in *best (nullable); *best_ms
 * (nullable) is its time per call (-1 when read from the file).  Synchronous; allocates the
 * candidates' scratch and one logL buffer. */
lt_status lt_autotune(lt_ctx* ctx, const double* params, int64_t batch, const lt_wf_cfg* cfg, const lt_grid* grid,
                      const lt_orbit* orbit, const lt_tdi_cfg* tdi, const lt_psd* psd, const lt_data* data,
                      const char* cache_path, int reps, lt_tuning* best, double* best_ms, void* stream);

/* Co-precessing modes h_lm(t_k) for the modes in cfg->mode_mask (ascending bit
 * order: 22, 21, 33, 32, 44), m > 0, zero before the f_low start (Sec. II.A).
 * modes: device complex FP64 [batch][n_modes][n] interleaved (re, im).
 * cfg->precision is ignored (always FP64). */
lt_status lt_phenomt_modes(lt_ctx* ctx, const double* params, int64_t batch, const lt_wf_cfg* cfg,
                           const lt_grid* grid, double* modes, void* stream);

/* Polarisations h+, hx on the grid via the single-sum twist-up of Eq. (2.4)
 * with the composite quaternion of Eqs. (2.5)-(2.6), times exp(2 i psi).
 * hpc: device FP64 [batch][2][n] (h+, then hx). */
lt_status lt_phenomt_polarizations(lt_ctx* ctx, const double* params, int64_t batch, const lt_wf_cfg* cfg,
                                   const lt_grid* grid, double* hpc, void* stream);

/* TDI response (Eqs. 2.7-2.11): link responses at the six links with delays
 * along the orbit, K-tap Lagrange interpolation at delayed times, TDI X, Y, Z
 * and A, E, T.  out: device [batch][3][n], double (LT_FP64) or float
 * (LT_MIXED).  status: nullable device int32 [batch]. */
lt_status lt_lisa_tdi_response(lt_ctx* ctx, const double* params, int64_t batch, const lt_wf_cfg* cfg,
                               const lt_grid* grid, const lt_orbit* orbit, const lt_tdi_cfg* tdi,
                               void* out, int32_t* status, void* stream);

/* Log-likelihood (Eq. 2.12 read with the sign of its footnote):
 *   logl[b]      = sum_c [(d_c|h_c) - (h_c|h_c)/2]
 *   logl_full[b] = -1/2 sum_c (h_c - d_c | h_c - d_c) = logl[b] - dd/2
 * with (a|b) = 4 df Re sum_{band} a~ conj(b~) / S (Eq. 2.13), a~ = dt * DFT.
 * Computed as -(r|r)/2 + dd/2 with the residual r = h - d formed in the time
 * domain.  logl, logl_full (nullable, not both): device FP64 [batch]; status
 * (nullable): device int32 [batch], written per template: 0 ok, 1 unphysical
 * parameters, 2 non-finite result, 3 the template's delayed reads spread over
 * more samples than the response kernel's window holds (a grid step far below
 * the orbit's light times); any nonzero status gives logL = logl_full = -inf.
 * Every launch runs on `stream`, in chunks of templates, so the call can be
 * captured into a HIP graph; a template's results do not depend on the batch
 * it came in or the chunk size.
 * Memory: workspace (nullable) is caller-owned device memory of
 * workspace_bytes, used for every per-call array (see lt_workspace_size); the
 * call then allocates and synchronises nothing, except that the first call
 * with a new grid length or orbit builds that grid's FFT plan and orbit node
 * table in the context (host work, an upload, kept for later calls).  The
 * chunk is the largest (up to the context's launch-shape chunk, 256 templates
 * unless lt_ctx_set_tuning or lt_autotune set another) that fits the
 * workspace; one smaller than a single template's needs is LT_ERR_WORKSPACE.
 * With workspace = null the context keeps its own scratch, grown on demand
 * (growth synchronises the device before the old block is freed) to full chunks:
 * 5 series of n samples per template of a chunk plus the tables, and the set-up
 * constants of every template of the call (624 bytes and a status word each; they are
 * computed for the whole batch in one launch).  The workspace, like the
 * context's scratch, is in use until the stream reaches the end of the call:
 * calls sharing a workspace or a context must be ordered (same stream, or
 * synchronised by the caller). */
lt_status lt_tdi_loglike(lt_ctx* ctx, const double* params, int64_t batch, const lt_wf_cfg* cfg,
                         const lt_grid* grid, const lt_orbit* orbit, const lt_tdi_cfg* tdi,
                         const lt_psd* psd, const lt_data* data, double* logl, double* logl_full,
                         int32_t* status, void* workspace, size_t workspace_bytes, void* stream);

/* lt_tdi_loglike for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same computation and
 * results, with every per-call array in a fixed scratch of 128 MiB that the library holds on
 * each GPU it runs on until the process ends.  The call allocates, frees and synchronises
 * nothing and records no events; the FFT plan and orbit node table for (grid, orbit) must
 * already be in the context (any lt_tdi_loglike call with them builds both), else
 * LT_ERR_CONFIG.  Templates run in chunks that fit the scratch (at 2^20 samples four in mixed
 * precision, two in FP64, beside the set-up constants of the whole batch); a batch and grid
 * for which chunks of one template do not fit return LT_ERR_WORKSPACE before any launch.  Every call on a GPU uses that GPU's one scratch, so
 * calls that overlap on one GPU (different streams or contexts, unsynchronised) race and give
 * wrong results: order them. */
lt_status lt_tdi_loglike_noalloc(lt_ctx* ctx, const double* params, int64_t batch, const lt_wf_cfg* cfg,
                                 const lt_grid* grid, const lt_orbit* orbit, const lt_tdi_cfg* tdi,
                                 const lt_psd* psd, const lt_data* data, double* logl, double* logl_full,
                                 int32_t* status, void* stream);

/* Workspace of lt_tdi_loglike for `batch` templates with this configuration:
 * bytes (nullable) for full-size chunks (min(batch, the context's chunk) templates per chunk),
 * min_bytes (nullable) for chunks of one template (both include the set-up constants of all
 * `batch` templates).  Host only; no device work. */
lt_status lt_workspace_size(lt_ctx* ctx, int64_t batch, const lt_wf_cfg* cfg, const lt_grid* grid,
                            const lt_tdi_cfg* tdi, size_t* bytes, size_t* min_bytes);

/* sum over the enabled channels of (x_c|x_c) (Eq. 2.13) for time series x
 * [batch][3][n] (double if precision == LT_FP64, else float); out: device FP64
 * [batch].  With x = the injection this is (d|d) = SNR^2. */
lt_status lt_noise_inner(lt_ctx* ctx, const void* x, int64_t batch, const lt_grid* grid, const lt_psd* psd,
                         int channels, int precision, double* out, void* stream);

/* Real-to-complex FFT times dt of rows [rows][n] (double or float by
 * precision) into spectra [rows][n/2+1] complex (same real type).  n must be
 * even with n/2 = n1 * n2, n1, n2 <= 1024 built from the radices 2, 3, 4, 5, 8. */
lt_status lt_rfft(lt_ctx* ctx, const void* x, int64_t rows, int64_t n, double dt, int precision, void* spec,
                  void* stream);

/* Analytic PSD of Eqs. (2.14)-(2.15) (readings: x = 2 pi f L / c,
 * acceleration noise 2.4e-15 m s^-2 / sqrt(Hz), TDI 2.0 factor 4 sin^2(2x)) on
 * the rfft grid of `grid`; bin 0 is set to +inf.  S: device FP64 [3][n/2+1].  A set-up
 * call: the spectra are computed on the host and copied on `stream`, and the call returns
 * after the copy (it synchronises the stream). */
lt_status lt_psd_sangria(const lt_grid* grid, int generation, double arm_m, double* S, void* stream);

/* Per-kernel timing for benchmarks: when enabled, the library records HIP
 * events around each launch on the launch stream.  lt_profile_read returns,
 * for kernel class k (0 per-template setup and the per-call tables, 1 response
 * kernel, 2 fft pass 1, 3 fft pass 2 + band reduction, 4 finalize, 5 waveform),
 * the summed milliseconds and launch counts since the last reset (it
 * synchronises the recorded events); n_classes <= 8. */
lt_status lt_profile_enable(lt_ctx* ctx, int on);
lt_status lt_profile_read(lt_ctx* ctx, double* ms, int64_t* launches, int n_classes);


/* ------------------------------------------------------------------------
 * On-device parallel-tempered ensemble sampler (Sec. II.C: the paper runs
 * ptemcee with Fisher-initialised walkers; here every step -- stretch-move
 * proposals, prior, batched logL, Metropolis-Hastings acceptance and the
 * adjacent-temperature swaps -- runs on the GPU and is replayed as one HIP
 * graph).  Random numbers: Philox4x32-10 keyed by the seed, counter
 * (step, purpose, slot, lane); one step needs no host interaction.
 *
 * Sampling coordinates (param_kind):
 *   LT_PARAMS_ALIGNED10:     m1, m2, chi1z, chi2z, D_L[Mpc], iota, phi_ref, beta, lambda, psi
 *   LT_PARAMS_PRECESSING14:  m1, m2, a1, theta1, phi1, a2, theta2, phi2, D_L[Mpc], iota, phi_ref,
 *                            beta, lambda, psi   (spins in polar form, Tab. I)
 *   LT_PARAMS_RAW:           the coordinates themselves (analytic test targets)
 * Priors are uniform boxes [lo, hi] (Tab. I; beta in [-pi/2, pi/2]).
 * Targets: LT_TARGET_TDI (lt_tdi_loglike with the stored configuration and
 * data), LT_TARGET_GAUSS (n_gauss Gaussians sharing one inverse covariance,
 * equal weights; for tests of the sampler itself). */
enum { LT_PARAMS_ALIGNED10 = 0, LT_PARAMS_PRECESSING14 = 1, LT_PARAMS_RAW = 2 };
enum { LT_TARGET_TDI = 0, LT_TARGET_GAUSS = 1 };

typedef struct lt_sampler lt_sampler;
typedef struct {
  int n_walkers;      /* per temperature; even, >= 4 */
  int n_temps;        /* >= 1; geometric ladder beta_i = t_max^(-i/(n_temps-1)) */
  int dim;            /* coordinates per walker (<= 32) */
  int param_kind;     /* LT_PARAMS_* */
  int target;         /* LT_TARGET_* */
  double stretch_a;   /* stretch-move scale a > 1 (2.0) */
  double t_max;       /* hottest temperature (>= 1) */
  uint64_t seed;
  double t_c;         /* fixed SSB peak time for the TDI target [s] */
  const double* lo;   /* host [dim] */
  const double* hi;   /* host [dim] */
  int n_gauss;        /* LT_TARGET_GAUSS: 1 or 2 */
  const double* gauss_mean;  /* host [n_gauss][dim] */
  const double* gauss_icov;  /* host [dim][dim] */
} lt_sampler_cfg;

/* Creates a sampler with its own context (so that the captured graph owns its
 * scratch).  For LT_TARGET_TDI the likelihood configuration is copied; the
 * device arrays psd->S[] and data->aet must stay valid for the sampler's life.
 * That context's chunk is 256 templates, doubled while a chunk's residual
 * (3 n samples per template) stays within 128 MiB and the workspace for half
 * the ensemble within 4 GiB (512 at 2^14 samples); results do not depend on it. */
lt_status lt_sampler_create(int hip_device, const lt_sampler_cfg* cfg, const lt_wf_cfg* wf, const lt_grid* grid,
                            const lt_orbit* orbit, const lt_tdi_cfg* tdi, const lt_psd* psd, const lt_data* data,
                            lt_sampler** out);
lt_status lt_sampler_destroy(lt_sampler* s);
/* Sets every walker (host [n_temps][n_walkers][dim], temperature-major) and
 * evaluates its log-prior and logL; resets the step counter and statistics. */
lt_status lt_sampler_set_state(lt_sampler* s, const double* pos);
/* Runs n_steps sampler steps (each: two half-ensemble stretch updates, then
 * the tempering swaps) on `stream` by replaying the captured graph. */
lt_status lt_sampler_step(lt_sampler* s, int n_steps, void* stream);
/* Copies the state to host memory (synchronises): pos [T][W][dim], logl and
 * logp [T][W] (nullable), step (nullable); counters (nullable, int64 [4]):
 * accepted moves, proposed moves, accepted swaps, proposed swaps. */
lt_status lt_sampler_get_state(lt_sampler* s, double* pos, double* logl, double* logp, uint64_t* step,
                               int64_t* counters);

/* Fisher matrix for the initialisation of the sampler (Sec. II.C: starting
 * points drawn from N(theta_inj, Gamma^-1), Gamma from finite differences of
 * the likelihood).  In zero noise at the injection Gamma_ij = (d_i h | d_j h)
 * (Eq. 2.13 summed over the enabled channels), computed here with central
 * differences of the TDI response in the sampling coordinates of param_kind
 * (steps: host [dim] half-widths).  x0: host [dim]; gamma: host [dim][dim].
 * Synchronous; FP64 throughout. */
lt_status lt_fisher(lt_ctx* ctx, const double* x0, int param_kind, double t_c, const double* steps,
                    const lt_wf_cfg* cfg, const lt_grid* grid, const lt_orbit* orbit, const lt_tdi_cfg* tdi,
                    const lt_psd* psd, double* gamma);

/* Draws count starting points from N(x0, Gamma^-1) (host FP64): Gamma is
 * symmetrised and scaled to unit diagonal, C = D Gamma D with
 * D = diag(Gamma_ii^-1/2) (1 where Gamma_ii <= 0); the eigenvalues of C are
 * floored at reg * its max eigenvalue (near-degenerate directions of 22-only
 * models) and x = x0 + D V W^-1/2 z, which has covariance Gamma^-1 exactly
 * when no eigenvalue is floored.  Normal deviates from Philox4x32-10
 * (Box-Muller); draws outside [lo, hi] are redrawn (up to 64 times, then
 * clipped).  out: host [count][dim]. */
lt_status lt_fisher_draw(const double* x0, const double* gamma, int dim, const double* lo, const double* hi,
                         int64_t count, uint64_t seed, double reg, double* out);

/* ---------------------------------------------------------------------------
 * Learned proposal (Sec. II.A names machine-learning proposals as a reason to
 * keep the whole pipeline on the accelerator; the flow itself is this
 * library's design).  A RealNVP-style normalising flow over the sampling
 * coordinates:
 *   u = Lw^-1 (x - mu) (Lw lower triangular: diag(sigma) or a full factor such
 *   as the Cholesky factor of a sample covariance); for layer l = 0..L-1 the conditioning set A_l is the
 *   first floor(d/2) coordinates (even l) or the last floor(d/2) (odd l), B_l
 *   the rest; h1 = relu(W1 u_A + b1), h2 = relu(W2 h1 + b2), o = W3 h2 + b3,
 *   s = 3 tanh(o[0:|B|] / 3), t = o[|B|:2|B|], u_B <- u_B exp(s) + t;
 *   log q(x) = -|z|^2/2 - (d/2) log 2pi + sum_l sum s_l - sum log diag(Lw).
 * Parameters: FP32 host vector, per layer W1[H][|A|], b1[H], W2[H][H], b2[H],
 * W3[2|B|][H], b3[2|B|] (row-major), layers in order.  The GEMMs run on the
 * matrix cores with BF16 operands and FP32 accumulation; the coupling update,
 * log-determinants and log q are FP64 (a flow with W3 = b3 = 0 is the exact
 * identity).  Training: Adam (beta1 0.9, beta2 0.999, eps 1e-8) on the mean
 * negative log q.  A flow object may be used by one host thread at a time;
 * its buffers are shared by all its calls, so calls on different streams
 * must not overlap. */
typedef struct lt_flow lt_flow;

/* 2 <= dim <= 64, 1 <= n_layers <= 32, hidden in [8, 4096] and a multiple of
 * 8, 1 <= max_batch <= 2^20 rows per call.  Parameters start at zero (the
 * identity flow, mu = 0, sigma = 1).  Device memory: about
 * n_layers * max_batch * (12 hidden + 26 dim) bytes of activations. */
lt_status lt_flow_create(int hip_device, int dim, int n_layers, int hidden, int max_batch, lt_flow** out);
lt_status lt_flow_destroy(lt_flow* f);
/* Number of FP32 parameters (-1 for a null flow). */
int64_t lt_flow_num_params(const lt_flow* f);
/* Host params [num_params], mu and sigma [dim] (sigma > 0, Lw = diag(sigma)); resets Adam's
 * moments and step count.  Synchronous. */
lt_status lt_flow_set_params(lt_flow* f, const float* params, const double* mu, const double* sigma);
/* Whitening only: mu [dim] and Lw host [dim][dim] row-major, of which only
 * the lower triangle is read (diagonal > 0); the network weights and Adam's
 * state are kept.  Synchronous. */
lt_status lt_flow_set_whitening(lt_flow* f, const double* mu, const double* L);
/* Copies the FP32 master parameters to host memory.  Synchronous. */
lt_status lt_flow_get_params(lt_flow* f, float* params);
/* log q of n rows of x (device FP64 [n][dim]) into logq (device FP64 [n]). */
lt_status lt_flow_log_prob(lt_flow* f, const double* x, int64_t n, double* logq, void* stream);
/* Inverse pass: base samples z (device FP64 [n][dim], standard normal) ->
 * x (device FP64 [n][dim]) and log q(x) (device FP64 [n]). */
lt_status lt_flow_sample(lt_flow* f, const double* z, int64_t n, double* x, double* logq, void* stream);
/* Mean negative log q of the n rows of x (device) and its gradient with
 * respect to the parameters; logq (host FP64 [n], nullable) and grad (host
 * FP32 [num_params], nullable).  Synchronous; does not update the weights. */
lt_status lt_flow_loss_grad(lt_flow* f, const double* x, int64_t n, double* logq, float* grad);
/* `steps` Adam steps on minibatches of `batch` rows of x (device FP64
 * [n][dim]); step i uses rows (i batch + r) mod n, r < batch (shuffle x to
 * randomise).  batch <= max_batch. */
lt_status lt_flow_train(lt_flow* f, const double* x, int64_t n, int steps, int batch, double lr, void* stream);

/* Attaches a flow (nullable: detach) to a sampler.  With a flow attached each
 * sampler step adds, after the two stretch half-steps and before the swaps,
 * an independence Metropolis-Hastings move for every walker of the coldest
 * rung: y from the flow (base normals from Philox counter
 * (step, 0x400, walker, q), two Box-Muller pairs per counter), accepted with
 * log u < beta_0 (logL_y - logL_x) + (logP_y - logP_x) + log q(x) - log q(y),
 * u from counter (step, 0x500, walker, 0).  The flow's dim must equal the
 * sampler's and its max_batch be >= n_walkers; the flow must outlive the
 * sampler or be detached first.  Retraining the attached flow between
 * lt_sampler_step calls changes the proposal in place. */
lt_status lt_sampler_set_flow(lt_sampler* s, lt_flow* flow);
/* Symmetry fold of the flow move, for a target invariant under x_i -> x_i + period
 * (the polarisation angle psi with period pi: h carries exp(2 i psi), Eq. (2.6)).
 * The flow then works on folded coordinates: the sampler maps x_i into the window
 * [start, start + period) before evaluating log q(x), and a flow sample y whose y_i
 * lies in the window becomes one of its copies y_i + k period inside the prior range
 * [lo_i, hi_i], chosen uniformly with u from Philox counter (step, 0x600, walker, 0);
 * a sample outside the window is rejected.  Both densities carry the factor
 * 1 / (number of copies), so the acceptance above stays exact.  index = -1 removes
 * the fold; period must be positive and finite.  The flow should be trained on folded
 * samples.  Rebuilds the captured step on the next lt_sampler_step. */
lt_status lt_sampler_set_flow_fold(lt_sampler* s, int index, double period, double start);
/* Turns the flow move into a random walk in the flow's latent space (step > 0;
 * 0 restores independence proposals): z = f(x) for the (folded) cold position,
 * z' = z + step eps with eps standard normal from Philox counter (step, 0x700,
 * walker, q) (two Box-Muller pairs per counter), y = f^-1(z').  The latent walk is
 * symmetric, so the acceptance above holds with log q(x) - log N(z) in place of
 * log q(x) and log q(y) - log N(z') in place of log q(y) (the ratio of the flow's
 * Jacobians); the fold applies as before.  Rebuilds the captured step. */
lt_status lt_sampler_set_flow_walk(lt_sampler* s, double step);
/* Mixes the flow move with the plain stretch move (the learned proposal's rate p_flow): each
 * sampler step runs the flow move with probability p_flow in [0, 1], decided on the device by
 * u < p_flow with u from Philox counter (step, 0x800, 0, 0); a step without it proposes
 * nothing for it (its likelihood rows are unphysical and skipped).  The choice does not depend
 * on the state, and every move is an exact Metropolis-Hastings step, so the mixture keeps the
 * target.  1 (the default) runs the flow move every step; 0 is the plain sampler (the
 * fallback), even with a flow attached.  Rebuilds the captured step. */
lt_status lt_flow_set_mix(lt_sampler* s, double p_flow);
/* on = 1: a step that runs the flow move (above) skips the stretch moves of the cold rung,
 * whose walkers then move by the flow move alone on that step (their stretch rows are neither
 * evaluated nor counted); the hotter rungs keep theirs.  The choice is the step's gate, not the
 * state, so the target is kept.  It saves the cold rung's likelihood rows on the flow's steps.
 * 0 (the default): both moves run.  Rebuilds the captured step.  Status LT_ERR_CONFIG unless
 * on is 0 or 1. */
lt_status lt_sampler_set_flow_exclusive(lt_sampler* s, int on);
/* A second flow for the flow move (second = NULL: one flow again): the independence proposal
 * becomes the mixture q = w_first q1 + (1 - w_first) q2, for posteriors with two modes (one
 * flow trained on each).  Each cold walker draws its component, the first flow when u < w_first
 * with u from Philox counter (step, 0x900, walker, 0); both flows map the step's base normals
 * and the walker takes its component's point; log q of the proposal and of the current (folded)
 * position is log(w_first q1 + (1 - w_first) q2), from both flows' forward passes, so the
 * acceptance above stays exact for q.  Same dimension, device and max_batch >= n_walkers as the
 * first flow; w_first in (0, 1); not with the latent walk (LT_ERR_CONFIG).  Like the first flow,
 * the second must outlive the sampler or be detached first.  Rebuilds the captured step. */
lt_status lt_sampler_set_flow_mixture(lt_sampler* s, lt_flow* second, double w_first);
/* Flow moves accepted and proposed since lt_sampler_set_state (host int64 [2]). */
lt_status lt_sampler_flow_counts(lt_sampler* s, int64_t* counts);

#ifdef __cplusplus
}
#endif
#endif
