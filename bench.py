"""Throughput of the time-domain LISA log-likelihood on one MI355X.

Workload (one "step" = one lt_tdi_loglike call over a batch, i.e. every hot
path step a1-a10 for every template of the batch): precessing spins with the
five co-precessing modes (2,2),(2,1),(3,3),(3,2),(4,4) twisted up, 2^20
samples at 5 s (~2 months), Keplerian unequal arms, TDI 2.0, A, E, T,
8-tap Lagrange interpolation at delayed times, mixed precision (FP64 phase,
time, orbit and sums; FP32 response and FFT), a batch of 256 templates of
uneven lengths (each starting at its own 0.1 mHz), zero-noise Tab. I
precessing injection as data.

Prints one JSON line (see the design notes for the roofline accounting).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Device counters of the bench configuration per template of a launch (a launch's counters
# scale with its templates), from rocprofv3 --pmc runs of this script (summaries in profiles/):
# HBM bytes (FETCH_SIZE, WRITE_SIZE scaled by the same process's 1 GiB copy calibration) and
# issued VALU wave-instructions (all, FP32 and FP64 multiply-adds), keyed by (kernel class,
# samples, taps, precision).  Any other configuration, or a kernel changed since the counters
# were taken, reports null.
PMC = {
    # profiles/k_tdi_precessing_k8_2p20_b256.md (a launch of 256 templates, divided by 256)
    ("tdi_response", 2 ** 20, 8, "mixed"): {"fetch": 2771580000 / 256, "write": 3221230000 / 256,
                                            "valu": 5.100e9 / 256, "fma_f32": 1.566e9 / 256, "fma_f64": 9.94e8 / 256},
    ("waveform", 2 ** 20, 8, "mixed"): {"fetch": 2473600 / 256, "write": 2147480000 / 256, "valu": 1.3455e9 / 256,
                                        "fma_f32": 3.4925e8 / 256, "fma_f64": 7.308e7 / 256},
}


def pmc_per_launch(kernel, n, taps, precision, templates):
    """The counters of one launch of `templates` templates (None when not profiled)."""
    v = PMC.get((kernel, n, taps, precision))
    return {k: x * templates for k, x in v.items()} if v and templates else {}

N_SAMPLES = 2 ** 20
BATCH = 256
TAPS = 8      # the smallest order whose interpolation error is below the FP32 floor (tests/test_oracle_taps.py)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=BATCH)
    ap.add_argument("--n", type=int, default=N_SAMPLES)
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--coarse", type=int, choices=[1, 2], default=1,
                    help="2: waveform on every second sample, linear in between (paper's 10 s -> 5 s)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=3)
    ap.add_argument("--no-sampler", action="store_true", help="skip the sampler-step and ESS measurements")
    ap.add_argument("--no-ess-precessing", action="store_true",
                    help="skip the ESS/s measurement on the precessing 14-D posterior (the C4 injection)")
    ap.add_argument("--p-flow", type=float, default=1.0,
                    help="fraction of sampler steps that run the flow move in the ESS measurements")
    ap.add_argument("--ess-reference", type=int, default=0,
                    help="with --ess-only: also run a plain chain of this many steps as the accuracy reference")
    ap.add_argument("--ess-only", choices=["aligned", "precessing"], default=None,
                    help="only run the ESS/s measurement of learned against plain proposals on that posterior")
    ap.add_argument("--flow-train", type=int, default=0, metavar="STEPS",
                    help="only time STEPS Adam steps of the flow (14-D, 8 couplings, width 256, batch 2048)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (known traffic) to calibrate HBM counters")
    return ap.parse_args()


SLICE = 1 << 17


def _oracle_time(args):
    """Seconds per template of the oracle (as it stands), on one core: the full chain
    (polarisations, six links, TDI 2.0 X, Y, Z, A, E, T) for one template on a contiguous
    slice of the grid, scaled to the whole grid, plus the rfft and band inner products of one
    full-length 3-channel series."""
    p, g, taps = args
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import likelihood as olk
    from oracle.orbits import Orbit
    from oracle.response import Response
    from oracle.waveform import Template
    with threadpool_limits(1):          # numpy's thread pools pinned: one core per process
        n = g["n"]
        r = Response(Template(p), g["t0"], g["dt"], n, Orbit("kepler"), taps=taps, precessing=True, generation=20)
        idx = np.arange(n - SLICE - 4096, n - 4096)
        t0 = time.perf_counter()
        r.aet(idx)
        t_resp = time.perf_counter() - t0
        x = np.random.default_rng(0).standard_normal((3, n))
        S = olk.channel_psds(n, g["dt"], 20)
        t0 = time.perf_counter()
        olk.loglike(x, 0.5 * x, S, g["dt"])
        t_fft = time.perf_counter() - t0
    return t_resp * (n / SLICE) + t_fft, t_resp + t_fft


def cpu_baseline(g, params, taps):
    """The oracle timed on the host's cores: one process per core (at most 16, the host share of
    one GPU), each running the bounded sample of _oracle_time on its own template, all at once;
    throughput = sum over processes of 1 / (seconds per template).  Also the same sample on
    one core alone."""
    import multiprocessing as mp
    single, work1 = _oracle_time((params[0], g, taps))
    P = max(1, min(os.cpu_count() or 1, 16))
    ctx = mp.get_context("spawn")       # fresh interpreters: nothing of this process's GPU state
    t0 = time.perf_counter()
    with ctx.Pool(P) as pool:
        res = pool.map(_oracle_time, [(params[i % len(params)], g, taps) for i in range(P)])
    wall = time.perf_counter() - t0
    value = sum(1.0 / per for per, _ in res)
    return {"value": value, "unit": "logL evals/s", "cores": P, "kind": "oracle",
            "sample": "oracle, one process per core on %d of the bench templates: response+TDI on %d of %d "
                      "samples (scaled x%.0f) + full-length rfft/inner products; %.1f s of work per process, "
                      "%.1f s wall" % (P, SLICE, g["n"], g["n"] / SLICE, max(w for _, w in res), wall),
            "single_core": {"value": 1.0 / single, "cores": 1, "seconds_measured": work1}}


# eigenvalue floor of the Fisher draws, relative to the largest eigenvalue of the unit-diagonal
# Fisher matrix (lt_fisher_draw): near-degenerate directions start at most 1000 times wider than
# the conditional widths.  At 1e-12 the precessing start spreads over the prior box and 2100
# burn-in steps leave the chains far from equilibrium (autocorrelation times near 100 steps)
FISHER_REG = 1e-6
FISHER_STEPS_P14 = [1.0, 1.0, 1e-4, 1e-4, 1e-4, 1e-4, 1e-4, 1e-4, 1.0, 1e-5, 1e-5, 1e-5, 1e-5, 1e-5]


def _tdi_setup(lib, inputs, ctx, n, prec, before_end=2000.0):
    """Precessing Tab. I injection (zero noise) on an n-sample grid: config, data, PSD, dd."""
    import torch
    dev = "cuda:0"
    g = inputs.grid(n, 5.0)
    modes = ((2, 2), (2, 1), (3, 3), (3, 2), (4, 4))
    cfg = ctx.wf_cfg(modes, True, precision=prec)
    cfg64 = ctx.wf_cfg(modes, True, precision=lib.LT_FP64)
    orb = ctx.orbit("kepler")
    tdi = ctx.tdi_cfg(20, 7, TAPS)
    S = torch.zeros((3, n // 2 + 1), dtype=torch.float64, device=dev)
    lib.psd_sangria(g, 20, S)
    inj = inputs.tab1_injection(True, g, before_end=before_end)
    d = torch.zeros((1, 3, n), dtype=lib.real_dtype(prec), device=dev)
    ctx.lisa_tdi_response(torch.tensor(inj[None], device=dev), g, cfg, orb, tdi, d)
    dd = torch.zeros(1, dtype=torch.float64, device=dev)
    ctx.noise_inner(d, g, S, dd, precision=prec)
    torch.cuda.synchronize()
    return dict(g=g, cfg=cfg, cfg64=cfg64, orb=orb, tdi=tdi, S=S, inj=inj, d=d, dd=float(dd.item()))


def _sampler(lib, inputs, ctx, su, W, T, seed):
    """Fisher-initialised sampler on the precessing 14-D coordinates."""
    x0, lo, hi = inputs.tab1_prior(True, su["inj"])
    G = lib.fisher(ctx, x0, "precessing14", su["inj"][11], FISHER_STEPS_P14, su["g"], su["cfg64"], su["orb"],
                   su["tdi"], su["S"])
    start = lib.fisher_draw(x0, G, lo, hi, T * W, seed, FISHER_REG)
    smp = lib.Sampler(W, T, 14, lo, hi, seed, target="tdi", param_kind="precessing14", t_c=su["inj"][11],
                      g=su["g"], cfg=su["cfg"], orbit=su["orb"], tdi=su["tdi"], psd=su["S"], data_aet=su["d"][0],
                      dd=su["dd"])
    smp.set_state(start)
    return smp


def sampler_bench(lib, inputs, prec, steps=200, W=512, T=8, ref_steps=10):
    """One full sampler step on the device (propose, waveform, response, FFT,
    logL, accept, swaps) replayed as a HIP graph: 512 walkers x 8 temperatures,
    precessing 14-D, 2^20 samples, TDI-2 AET, Fisher-initialised; `steps` steps timed,
    and the likelihood alone (two calls of half the ensemble) over `ref_steps`."""
    import torch
    ctx = lib.Context(0)
    su = _tdi_setup(lib, inputs, ctx, N_SAMPLES, prec)
    smp = _sampler(lib, inputs, ctx, su, W, T, 11)
    smp.step(1)                                    # captures the graph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    smp.step(steps)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    _, _, _, k, cnt = smp.state()
    smp.close()
    # the likelihood alone: two calls of T W / 2 templates a step (the step's two half-ensembles),
    # templates next to the injection (every one spans the whole grid, as the walkers' do)
    import numpy as np
    rng = np.random.default_rng(12)
    P = np.repeat(su["inj"][None], T * W // 2, axis=0)
    P[:, 0] *= 1.0 + 1e-5 * rng.standard_normal(T * W // 2)
    P[:, 1] *= 1.0 + 1e-5 * rng.standard_normal(T * W // 2)
    params = torch.tensor(P, device="cuda:0")
    out = torch.zeros(T * W // 2, dtype=torch.float64, device="cuda:0")

    def half():
        ctx.tdi_loglike(params, su["g"], su["cfg"], su["orb"], su["tdi"], su["S"], su["d"][0], su["dd"], out)

    half()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(2 * ref_steps):
        half()
    torch.cuda.synchronize()
    dl = (time.perf_counter() - t0) / ref_steps
    ctx.close()
    return {"walkers": W, "temps": T, "steps": steps, "ms_per_step": 1e3 * dt, "steps_per_s": 1.0 / dt,
            "logl_per_s": T * W / dt, "stretch_accept": cnt[0] / max(cnt[1], 1),
            "swap_accept": cnt[2] / max(cnt[3], 1), "loglike_only_ms_per_step": 1e3 * dl,
            "overhead_ms_per_step": 1e3 * (dt - dl)}


FISHER_STEPS_A10 = [1.0, 1.0, 1e-4, 1e-4, 1.0, 1e-5, 1e-5, 1e-5, 1e-5, 1e-5]


def _record(smp, k):
    import numpy as np
    chain = []
    for _ in range(k):
        smp.step(1)
        chain.append(smp.state()[0][0].copy())
    return np.array(chain)


def flow_gemm_flops(d, layers=8, hidden=256):
    """Matrix-core work of one training sample of the flow: per coupling the products with
    W1[H][|A|], W2[H][H] and W3[2|B|][H] (|A| = floor(d/2), |B| = d - |A|), 2 flops per
    multiply-add, three times over (forward, input gradients, weight gradients)."""
    a = d // 2
    return 3 * layers * 2 * (hidden * a + hidden * hidden + 2 * (d - a) * hidden)


def split_modes(s, min_sep=8.0, min_frac=0.02, axes=4):
    """The larger of two clusters of s when s holds two well separated modes (a boolean mask of
    its rows), else None.  Two-means on coordinates scaled by their standard deviations,
    started from a split at the median along each of the first `axes` principal axes; the best
    separated split counts when the Mahalanobis distance between its means under the pooled
    within-cluster covariance is at least min_sep (a median split of one Gaussian gives about
    2.7) and its smaller part holds at least min_frac of the samples."""
    import numpy as np
    z = (s - s.mean(0)) / s.std(0)
    vt = np.linalg.svd(z, full_matrices=False)[2]
    best, best_sep = None, 0.0
    for a in range(min(axes, z.shape[1])):
        p = z @ vt[a]
        lab = p > np.median(p)
        for _ in range(50):
            new = ((z - z[lab].mean(0)) ** 2).sum(1) < ((z - z[~lab].mean(0)) ** 2).sum(1)
            if np.array_equal(new, lab) or new.all() or not new.any():
                break
            lab = new
        if lab.all() or not lab.any():
            continue
        d = z[lab].mean(0) - z[~lab].mean(0)
        f = lab.mean()
        sw = f * np.cov(z[lab].T) + (1.0 - f) * np.cov(z[~lab].T)
        sep = float(np.sqrt(d @ np.linalg.solve(sw, d)))
        if sep > best_sep:
            best, best_sep = lab, sep
    if best is None or best_sep < min_sep or min(best.mean(), 1.0 - best.mean()) < min_frac:
        return None
    return best if best.mean() >= 0.5 else ~best


def dominant_mode(s, min_sep=8.0, min_frac=0.02, axes=4):
    """The samples of the more populated of two clusters when s holds two well separated modes,
    else all of s; and the fraction kept (split_modes)."""
    keep = split_modes(s, min_sep, min_frac, axes)
    if keep is None:
        return s, 1.0
    return s[keep], float(keep.mean())


def quantile_gap(a, b, n_batches=20):
    """Largest difference between the 5 / 50 / 95 % marginal quantiles of two chains
    [steps][walkers][d], in units of its Monte-Carlo standard error (batch quantiles)."""
    import numpy as np
    from paper_2501_08261_amd.diagnostics import batch_quantile_se
    qa, sa = batch_quantile_se(a, n_batches=n_batches)
    qb, sb = batch_quantile_se(b, n_batches=n_batches)
    return float(np.max(np.abs(qa - qb) / np.sqrt(sa ** 2 + sb ** 2)))


def train_early_stop(flow, s, mu, L, val_frac=0.25, chunk=250, max_steps=3000, patience=1, lr=3e-4, seed=0):
    """Fit the flow to a window of chain samples s [n][d] in time order, holding out its last
    val_frac of rows: Adam in chunks of `chunk` steps (batch 2048) on the shuffled earlier
    samples, the held-out mean log q after each chunk, stop after `patience` chunks without
    improvement and keep the best parameters.  The chain is correlated in time, so a later
    stretch of it is the fair check of what the flow will meet as a proposal; training on
    without it overfits the window (the held-out log q falls while the training one rises).
    Returns (Adam steps run, best held-out mean log q)."""
    import numpy as np
    import torch
    nv = max(1, int(round(val_frac * s.shape[0])))
    tr = s[:-nv]
    va = torch.tensor(s[-nv:], device="cuda:0")
    flow.set_whitening(mu, L)
    xs = torch.tensor(tr[np.random.default_rng(seed).permutation(len(tr))], device="cuda:0")

    def val_logq():
        tot = 0.0
        for i in range(0, va.shape[0], flow.max_batch):
            tot += float(flow.log_prob(va[i:i + flow.max_batch]).sum().item())
        return tot / va.shape[0]
    best, best_p, bad, done = val_logq(), flow.get_params(), 0, 0
    while done < max_steps and bad < patience:
        # each chunk starts where the previous one stopped in the shuffled samples
        flow.train(torch.roll(xs, -((done * 2048) % xs.shape[0]), 0), chunk, 2048, lr)
        done += chunk
        v = val_logq()
        if v > best:
            best, best_p, bad = v, flow.get_params(), 0
        else:
            bad += 1
    flow.set_params(best_p, np.zeros(s.shape[-1]), np.ones(s.shape[-1]))
    flow.set_whitening(mu, L)
    return done, best


def ess_bench(lib, inputs, prec, precessing=False, n=1 << 14, W=512, T=8, burn=500, rounds=4, window=400,
              train_steps=1500, m=1000, walk=0.0, modes="mixture", p_flow=1.0, early_stop=True, pool=1,
              exclusive=True, control=True, reinit=False, fisher_reg=None, ref_steps=0):
    """Effective samples per second of the cold chain, stretch moves alone against
    stretch + learned-flow moves, on one injection and one GPU (TDI-2 AET, 512
    walkers x 8 temperatures, n samples around the merger, Fisher-initialised).

    The flow (8 couplings, width 256) learns from the sampler's own chain: after
    `burn` plain steps, `rounds` times: take the cold samples of the last `pool` windows
    of `window` steps, whiten by the Cholesky factor of their covariance, train on them
    (train_early_stop: at most `train_steps` Adam steps, stopped by the latest quarter of
    the samples; early_stop=False: exactly `train_steps`), attach, run `window` more steps.
    When the samples hold two separated modes (split_modes), modes="mixture" trains one flow
    on each and proposes from their mixture, weighted by the modes' shares
    (lt_sampler_set_flow_mixture); modes="dominant" trains on the larger mode only; "off"
    trains on everything.  The flows are then frozen and both samplers
    restart from the same state for `m` recorded steps; ESS = m W / max_q tau_q
    (worst coordinate), ESS/s uses the time of 200 unrecorded steps.

    The waveform carries exp(2 i psi), so the likelihood is invariant under
    psi -> psi + pi and the prior range [-pi, pi] holds two copies of every psi.
    The flow works on psi folded into a window of width pi centred on the chain's
    circular mean of 2 psi (lt_sampler_set_flow_fold); its proposals land on either
    copy.  Autocorrelation times and moments are computed on the folded psi for both
    chains, since only psi mod pi is identified.

    walk > 0 replaces the flow's independence proposals by a random walk of that step in
    its latent space (lt_sampler_set_flow_walk).  p_flow < 1 runs the flow move on that
    fraction of the steps once the flow is attached (lt_flow_set_mix); the others run the
    stretch moves and swaps alone.  exclusive: the flow's steps skip the cold rung's stretch
    moves (lt_sampler_set_flow_exclusive).  control: also compare two plain chains.  reinit:
    each round trains a freshly initialised flow instead of continuing the last one.
    fisher_reg: the eigenvalue floor of the Fisher start (None: FISHER_REG).  Posterior
    accuracy: the largest gap between the two chains' 5 / 50 / 95 % quantiles in units of its
    Monte-Carlo error (quantile_gap)."""
    import numpy as np
    import torch
    from paper_2501_08261_amd.diagnostics import autocorr_time, batch_ess
    kind = "precessing14" if precessing else "aligned10"
    modes = ((2, 2), (2, 1), (3, 3), (3, 2), (4, 4))
    ctx = lib.Context(0)
    g = inputs.grid(n, 5.0)
    cfg = ctx.wf_cfg(modes, precessing, precision=prec)
    cfg64 = ctx.wf_cfg(modes, precessing, precision=lib.LT_FP64)
    orb, tdi = ctx.orbit("kepler"), ctx.tdi_cfg(20, 7, TAPS)
    S = torch.zeros((3, n // 2 + 1), dtype=torch.float64, device="cuda:0")
    lib.psd_sangria(g, 20, S)
    inj = inputs.tab1_injection(precessing, g)
    d = torch.zeros((1, 3, n), dtype=lib.real_dtype(prec), device="cuda:0")
    ctx.lisa_tdi_response(torch.tensor(inj[None], device="cuda:0"), g, cfg, orb, tdi, d)
    dd = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    ctx.noise_inner(d, g, S, dd, precision=prec)
    x0, lo, hi = inputs.tab1_prior(precessing, inj)
    dim = x0.size
    G = lib.fisher(ctx, x0, kind, inj[11], FISHER_STEPS_P14 if precessing else FISHER_STEPS_A10, g, cfg64, orb,
                   tdi, S)
    smp = lib.Sampler(W, T, dim, lo, hi, 5, target="tdi", param_kind=kind, t_c=inj[11], g=g, cfg=cfg, orbit=orb,
                      tdi=tdi, psd=S, data_aet=d[0], dd=float(dd.item()))
    reg = FISHER_REG if fisher_reg is None else fisher_reg
    smp.set_state(lib.fisher_draw(x0, G, lo, hi, T * W, 5, reg))
    t0 = time.perf_counter()
    smp.step(burn)
    flow = lib.Flow(dim, 8, 256, max(2048, W))
    flow.set_params(lib.flow_init_params(dim, 8, 256, 3), np.zeros(dim), np.ones(dim))
    ipsi = dim - 1

    def fold(X, start):
        X = np.array(X, copy=True)
        X[..., ipsi] = start + np.mod(X[..., ipsi] - start, np.pi)
        return X

    flow2 = None
    t_train = 0.0
    mode_frac, steps_run, recent = [], [], []

    def fit_flow(f, rows, r):
        """train f on rows (time order); seconds and Adam steps"""
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if early_stop:
            # whitened by the earlier 3/4 of the rows, which it trains on; the latest quarter
            # decides when to stop
            fit = rows[:len(rows) - max(1, int(round(0.25 * len(rows))))]
            done, _ = train_early_stop(f, rows, fit.mean(0), np.linalg.cholesky(np.cov(fit.T)),
                                       max_steps=train_steps, seed=r)
        else:
            f.set_whitening(rows.mean(0), np.linalg.cholesky(np.cov(rows.T)))
            xs = torch.tensor(rows[np.random.default_rng(r).permutation(len(rows))], device="cuda:0")
            f.train(xs, train_steps, 2048, 3e-4)
            done = train_steps
        torch.cuda.synchronize()
        return time.perf_counter() - t1, done

    for r in range(rounds):
        recent.append(_record(smp, window).reshape(-1, dim))
        s = np.concatenate(recent[-pool:])
        two = 2.0 * s[:, ipsi]
        start = 0.5 * np.arctan2(np.sin(two).mean(), np.cos(two).mean()) - 0.5 * np.pi
        s = fold(s, start)
        keep = split_modes(s) if modes != "off" else None
        mode_frac.append(1.0 if keep is None else float(keep.mean()))
        smp.set_flow_fold(ipsi, np.pi, start)
        smp.set_flow_walk(walk)
        if reinit:
            flow.set_params(lib.flow_init_params(dim, 8, 256, 3 + r), np.zeros(dim), np.ones(dim))
        dt, done = fit_flow(flow, s if keep is None else s[keep], r)
        t_train += dt
        steps_run.append(done)
        if keep is not None and modes == "mixture":
            if flow2 is None:
                flow2 = lib.Flow(dim, 8, 256, max(2048, W))
                flow2.set_params(lib.flow_init_params(dim, 8, 256, 4), np.zeros(dim), np.ones(dim))
            dt, done = fit_flow(flow2, s[~keep], r)
            t_train += dt
            steps_run.append(done)
        smp.set_flow(flow)
        smp.set_flow_mixture(flow2 if (keep is not None and modes == "mixture") else None,
                             float(keep.mean()) if keep is not None else 0.5)
        smp.set_flow_mix(p_flow)
        smp.set_flow_exclusive(exclusive)
    _record(smp, window)
    t_adapt = time.perf_counter() - t0
    state = smp.state()[0]
    res, chains = {}, {}
    for label, fl in (("learned", flow), ("plain", None)):
        smp.set_state(state)
        smp.set_flow(fl)
        smp.step(20)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        smp.step(200)
        torch.cuda.synchronize()
        t_step = (time.perf_counter() - t1) / 200
        chain = fold(_record(smp, m), start)
        acc, prop = smp.flow_counts()
        tau = autocorr_time(chain)
        chains[label] = chain
        eb = batch_ess(chain)
        flat = chain.reshape(-1, dim)
        res[label] = {"ess_per_s": m * W / float(tau.max()) / (m * t_step), "tau_max": float(tau.max()),
                      "tau_median": float(np.median(tau)), "ms_per_step": 1e3 * t_step,
                      "ess_batch": float(eb.min()), "ess_batch_per_s": float(eb.min()) / (m * t_step),
                      "ess_batch_coord": [round(float(v)) for v in eb],
                      "mean": flat.mean(0), "std": flat.std(0)}
        if fl is not None:
            res[label]["flow_accept"] = acc / max(prop, 1)
        else:
            res[label]["stretch_accept"] = smp.state()[4][0] / max(smp.state()[4][1], 1)
    qgap_control = None
    ctrl_shift = ctrl_std = None
    if control:
        # a second plain chain from the same state with another seed: the gap two plain chains
        # show is the floor of the check
        smp2 = lib.Sampler(W, T, dim, lo, hi, 6, target="tdi", param_kind=kind, t_c=inj[11], g=g, cfg=cfg,
                           orbit=orb, tdi=tdi, psd=S, data_aet=d[0], dd=float(dd.item()))
        smp2.set_state(state)
        smp2.step(220)
        c2 = fold(_record(smp2, m), start)
        qgap_control = quantile_gap(c2, chains["plain"])
        f2 = c2.reshape(-1, c2.shape[-1])
        ctrl_shift = float(np.max(np.abs(f2.mean(0) - res["plain"]["mean"]) / res["plain"]["std"]))
        ctrl_std = (f2.std(0) / res["plain"]["std"]).tolist()
        smp2.close()
    reference = None
    if ref_steps > 0:
        # a long plain chain (another seed, every 10th step kept) as the reference that both
        # measured chains are held against: their means in its standard deviations, their
        # standard deviations over its own
        smp3 = lib.Sampler(W, T, dim, lo, hi, 7, target="tdi", param_kind=kind, t_c=inj[11], g=g, cfg=cfg,
                           orbit=orb, tdi=tdi, psd=S, data_aet=d[0], dd=float(dd.item()))
        smp3.set_state(state)
        smp3.step(220)
        rows = []
        for i in range(ref_steps // 10):
            smp3.step(10)
            rows.append(smp3.state()[0][0].copy())
            if (i + 1) % 200 == 0:
                print("reference chain: %d steps" % (10 * (i + 1)), file=sys.stderr, flush=True)
        smp3.close()
        fr = fold(np.array(rows), start).reshape(-1, dim)
        mr, sr = fr.mean(0), fr.std(0)
        reference = {"steps": ref_steps}
        for label, ch in (("learned", chains["learned"]), ("plain", chains["plain"])) + \
                ((("plain2", c2),) if control else ()):
            f = ch.reshape(-1, dim)
            reference[label] = {"mean_shift_sigma": float(np.max(np.abs(f.mean(0) - mr) / sr)),
                                "std_ratio": [round(float(x), 3) for x in f.std(0) / sr]}
    # with the flow's training counted: the learned sampler's wall time includes the Adam steps;
    # break-even = the number of measured steps after which the learned sampler with its
    # training has produced as many effective samples per second as the plain one
    for v in res.values():
        v["ess_per_step"] = W / v["tau_max"]
    rl, rp = res["learned"]["ess_per_step"], res["plain"]["ess_per_step"]
    tl, tp = 1e-3 * res["learned"]["ms_per_step"], 1e-3 * res["plain"]["ms_per_step"]
    res["learned"]["ess_per_s_with_training"] = m * rl / (m * tl + t_train)
    gain = rl * tp - rp * tl
    breakeven = rp * t_train / gain if gain > 0 else None
    sd = res["plain"]["std"]
    shift = float(np.max(np.abs(res["learned"]["mean"] - res["plain"]["mean"]) / sd))
    std_ratio = (res["learned"]["std"] / sd).tolist()
    # Fisher widths at the injection against the MCMC widths (the paper's Tabs. II-III compare
    # the two): sqrt(diag(Gamma^-1)), inverted in the basis where Gamma has a unit diagonal (the
    # coordinates span many orders of magnitude: masses in Msun beside angles), eigenvalues of
    # that correlation-like matrix floored at 1e-15 of the largest
    dg = np.sqrt(np.diag(G))
    ev, V = np.linalg.eigh(G / np.outer(dg, dg))
    ev = np.maximum(ev, 1e-15 * ev.max())
    sig_f = np.sqrt(np.diag((V / ev) @ V.T)) / dg
    names = (["m1", "m2", "a1", "theta1", "phi1", "a2", "theta2", "phi2"] if precessing else
             ["m1", "m2", "chi1z", "chi2z"]) + ["D_L", "iota", "phi_ref", "beta", "lambda", "psi"]
    fisher = {"names": names, "sigma_fisher": [float("%.4g" % v) for v in sig_f],
              "sigma_mcmc": [float("%.4g" % v) for v in sd],
              "mcmc_over_fisher": [round(float(v), 3) for v in sd / sig_f],
              "prior_width": [float("%.4g" % v) for v in (hi - lo)]}
    for v in res.values():
        del v["mean"], v["std"]
    smp.close()
    flow.close()
    if flow2 is not None:
        flow2.close()
    ctx.close()
    qgap = quantile_gap(chains["learned"], chains["plain"])
    return {"target": kind, "flow_move": "latent walk, step %g" % walk if walk > 0 else "independence",
            "p_flow": p_flow, "flow_exclusive": bool(exclusive), "quantile_gap_mc_sigma": qgap,
            "quantile_gap_plain_vs_plain": qgap_control,
            "n_samples": n, "walkers": W, "temps": T, "steps_measured": m,
            "flow_training_share": mode_frac, "modes": modes,
            "adaptive_burn_in_s": t_adapt, "flow_train_s": t_train, "train_steps": steps_run,
            "flow_train_tflops": flow_gemm_flops(dim) * 2048 * sum(steps_run) / t_train / 1e12,
            "plain": res["plain"], "learned": res["learned"],
            "ratio": res["learned"]["ess_per_s"] / res["plain"]["ess_per_s"],
            "ratio_batch": res["learned"]["ess_batch_per_s"] / res["plain"]["ess_batch_per_s"],
            "ratio_with_training": res["learned"]["ess_per_s_with_training"] / res["plain"]["ess_per_s"],
            "breakeven_steps": breakeven,
            "posterior_mean_shift_sigma": shift, "posterior_std_ratio": [round(x, 3) for x in std_ratio],
            "plain_vs_plain": None if ctrl_std is None else
            {"mean_shift_sigma": ctrl_shift, "std_ratio": [round(x, 3) for x in ctrl_std]},
            "against_long_plain_chain": reference,
            "fisher_vs_mcmc": fisher}


def mixed_vs_fp64(lib, inputs, ctx, g, P, modes, orb, tdi, S, coarse):
    """Per-result error of the mixed-precision likelihood against the FP64 path (which matches
    the oracle to 1e-6 + 1e-11 (d|d)), both on the same data: the FP64 zero-noise injection,
    rounded to FP32 for the mixed path, with (d|d) of the rounded series in FP64.  Templates:
    the bench batch, the injection itself and 15 templates next to it (relative offsets of
    1e-5 in the masses and 1e-4 in the angles)."""
    import numpy as np
    import torch
    dev = "cuda:0"
    n = g["n"]
    inj = inputs.tab1_injection(True, g)
    rng = np.random.default_rng(17)
    near = np.repeat(inj[None], 15, axis=0)
    near[:, 0:2] *= 1.0 + 1e-5 * rng.standard_normal((15, 2))
    near[:, 9:11] += 1e-4 * rng.standard_normal((15, 2))
    near[:, 12:15] += 1e-4 * rng.standard_normal((15, 3))
    Q = np.concatenate([P, inj[None], near])
    cfg64 = ctx.wf_cfg(modes, True, precision=lib.LT_FP64, coarse=coarse)
    cfg32 = ctx.wf_cfg(modes, True, precision=lib.LT_MIXED, coarse=coarse)
    d64 = torch.zeros((1, 3, n), dtype=torch.float64, device=dev)
    ctx.lisa_tdi_response(torch.tensor(inj[None], device=dev), g, cfg64, orb, tdi, d64)
    d32 = d64.float()
    dd = torch.zeros(1, dtype=torch.float64, device=dev)
    ctx.noise_inner(d32.double(), g, S, dd)
    torch.cuda.synchronize()
    ddv = float(dd.item())
    params = torch.tensor(Q, device=dev)
    l64 = torch.zeros(len(Q), dtype=torch.float64, device=dev)
    l32 = torch.zeros(len(Q), dtype=torch.float64, device=dev)
    ctx.tdi_loglike(params, g, cfg64, orb, tdi, S, d32.double()[0].contiguous(), ddv, l64)
    ctx.tdi_loglike(params, g, cfg32, orb, tdi, S, d32[0].contiguous(), ddv, l32)
    torch.cuda.synchronize()
    a64, a32 = l64.cpu().numpy(), l32.cpu().numpy()
    ok = np.isfinite(a64) & np.isfinite(a32)
    err = np.abs(a32 - a64)[ok]
    rel = (err / np.maximum(np.abs(a64[ok]), 1e-300))
    nb = len(P)
    return {"templates": int(len(Q)), "compared": int(ok.sum()), "max_abs": float(err.max()),
            "median_abs": float(np.median(err)), "max_rel": float(rel.max()),
            "injection_abs": float(abs(a32[nb] - a64[nb])),
            "near_injection_max_abs": float(np.max(np.abs(a32[nb + 1:] - a64[nb + 1:]))),
            "near_injection_logl_full_range": [float(np.min(a64[nb + 1:] - 0.5 * ddv)),
                                               float(np.max(a64[nb + 1:] - 0.5 * ddv))]}


def flow_train_bench(lib, steps, d=14, layers=8, hidden=256, batch=2048):
    """Adam steps of the flow on 20,000 standard-normal rows: ms per step and the matrix-core
    rate of its GEMMs (flow_gemm_flops per row)."""
    import numpy as np
    import torch
    f = lib.Flow(d, layers, hidden, batch)
    f.set_params(lib.flow_init_params(d, layers, hidden, 3), np.zeros(d), np.ones(d))
    x = torch.tensor(np.random.default_rng(0).standard_normal((20000, d)), device="cuda:0")
    f.train(x, 20, batch, 3e-4)
    torch.cuda.synchronize()
    t = time.perf_counter()
    f.train(x, steps, batch, 3e-4)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / steps
    f.close()
    return {"flow_train_ms_per_step": 1e3 * dt, "steps": steps, "batch": batch, "dim": d, "layers": layers,
            "hidden": hidden, "tflops": flow_gemm_flops(d, layers, hidden) * batch / dt / 1e12}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only (the library has no multi-GPU path); got --gpus %d" % a.gpus,
              file=sys.stderr)
        sys.exit(2)
    if a.flow_train > 0:
        from paper_2501_08261_amd import lib
        print(json.dumps(flow_train_bench(lib, a.flow_train)))
        return
    if a.ess_only:
        from paper_2501_08261_amd import inputs, lib
        prec = lib.LT_MIXED if a.precision == "mixed" else lib.LT_FP64
        r = ess_bench(lib, inputs, prec, precessing=a.ess_only == "precessing", p_flow=a.p_flow,
                      ref_steps=a.ess_reference)
        print(json.dumps(r, default=float))
        return
    import numpy as np
    import torch
    from paper_2501_08261_amd import inputs, lib
    dev = "cuda:0"
    prec = lib.LT_MIXED if a.precision == "mixed" else lib.LT_FP64
    rdt = lib.real_dtype(prec)
    g = inputs.grid(a.n, 5.0)
    ctx = lib.Context(0)
    modes = ((2, 2), (2, 1), (3, 3), (3, 2), (4, 4))
    cfg = ctx.wf_cfg(modes, True, precision=prec, coarse=a.coarse)
    orb = ctx.orbit("kepler")
    tdi = ctx.tdi_cfg(20, 7, TAPS)
    S = torch.zeros((3, a.n // 2 + 1), dtype=torch.float64, device=dev)
    lib.psd_sangria(g, 20, S)
    inj = inputs.tab1_injection(True, g)
    d = torch.zeros((1, 3, a.n), dtype=rdt, device=dev)
    ctx.lisa_tdi_response(torch.tensor(inj[None], device=dev), g, cfg, orb, tdi, d)
    dd = torch.zeros(1, dtype=torch.float64, device=dev)
    ctx.noise_inner(d, g, S, dd, precision=prec)
    torch.cuda.synchronize()
    P = inputs.draw_templates(3, a.batch, g, precessing=True)
    params = torch.tensor(P, device=dev)
    logl = torch.zeros(a.batch, dtype=torch.float64, device=dev)
    status = torch.zeros(a.batch, dtype=torch.int32, device=dev)
    ddv = float(dd.item())
    # active samples per template (each starts at its own f_low): the first nonzero sample of
    # its polarisations, from the library; the algorithmic work of samples before it is zero
    active = []
    hbuf = torch.zeros((32, 2, a.n), dtype=torch.float64, device=dev)
    for c0 in range(0, a.batch, 32):
        nb = min(32, a.batch - c0)
        ctx.phenomt_polarizations(params[c0:c0 + nb].contiguous(), g, ctx.wf_cfg(modes, True), hbuf[:nb])
        nz = (hbuf[:nb] != 0).any(dim=1)
        first = torch.where(nz.any(dim=1), nz.float().argmax(dim=1), torch.full((nb,), a.n, device=dev))
        active += (a.n - first).tolist()
    del hbuf
    active_frac = float(np.mean(active)) / a.n

    # launch shape (templates per launch, work order, persistent grid): chosen by the library's
    # autotuner on this workload, cached per workload in the temporary directory
    import tempfile
    tuning, tune_ms = ctx.autotune(params, g, cfg, orb, tdi, S, d[0], ddv,
                                   cache_path=os.path.join(tempfile.gettempdir(), "lisatd_tuning.txt"), reps=3)
    print("tuning %s (%.3f ms per call)" % (tuning, tune_ms), file=sys.stderr, flush=True)

    def step():
        ctx.tdi_loglike(params, g, cfg, orb, tdi, S, d[0], ddv, logl, status=status)

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    print("warmup done", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for _ in range(a.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / a.steps
    value = a.batch * a.steps / elapsed
    print("timed %d steps: %.3f ms/step" % (a.steps, ms_per_step), file=sys.stderr, flush=True)

    # per-kernel averages from HIP events that the library records around each launch on its
    # stream (every launch of the likelihood is on the caller's stream), over a few more steps
    ctx.profile_enable(True)
    for _ in range(a.profile_steps):
        step()
    torch.cuda.synchronize()
    ms, cnt = ctx.profile_read(6)
    ctx.profile_enable(False)
    names = ["setup", "tdi_response", "fft_pass1", "fft_pass2_band", "finalize", "waveform"]
    kern = {names[i]: {"avg_ms": ms[i] / max(cnt[i], 1), "launches": cnt[i]} for i in range(6)}
    n_ok = int((status == 0).sum().item())
    # roofline of the dominant kernel (algorithmic work per template-sample, design notes)
    rsz = 4 if prec == lib.LT_MIXED else 8
    fft_bytes = {"fft_pass1": 3 * 2 * rsz, "fft_pass2_band": 3 * rsz}      # per real sample, per template
    # the dominant kernel: largest time per step; the templates one launch processes follow
    # from its launch count (the likelihood runs in chunks)
    dom = max(kern, key=lambda k: kern[k]["avg_ms"] * kern[k]["launches"])
    for k in kern:
        kern[k]["templates_per_launch"] = a.batch * a.profile_steps / max(kern[k]["launches"], 1) \
            if k != "setup" else None
    per_launch = kern[dom]["templates_per_launch"]
    units = a.n * per_launch * (active_frac if dom == "tdi_response" else 1.0)   # template-samples of work
    pmc = pmc_per_launch(dom, a.n, TAPS, a.precision, per_launch)
    traffic = pmc["fetch"] + pmc["write"] if "fetch" in pmc else None
    t_dom = kern[dom]["avg_ms"] * 1e-3
    if dom in fft_bytes:
        achieved = fft_bytes[dom] * units / t_dom / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": 8000.0, "unit": "GB/s", "frac": achieved / 8000.0,
                "traffic": traffic, "kernel": dom}
    else:
        from paper_2501_08261_amd import workcount
        flops = workcount.tdi_flops_per_sample(TAPS, 20)
        achieved = flops * units / t_dom / 1e12
        # one multiply-add per lane per clock: 256 CUs x 64 lanes x 2 flops x 2.4 GHz (the build
        # emits no packed FP32 instructions, so the FP32 ceiling is the FP64 one)
        peak = workcount.VALU_PEAK_TFLOPS
        roof = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": traffic, "kernel": dom,
                "achieved_is": "algorithmic-equivalent: the direct method's %d flops per active template-sample "
                               "(combined filters execute fewer)" % flops}
        if "fma_f32" in pmc:
            ex = workcount.executed_flops(pmc["fma_f32"], pmc["fma_f64"])
            roof["executed"] = {"tflops": ex / t_dom / 1e12, "frac": ex / t_dom / 1e12 / peak,
                                "valu_insts_per_cycle_per_cu": workcount.issue_rate(pmc["valu"], t_dom),
                                "source": "SQ_INSTS_VALU_FMA_F32/F64, SQ_INSTS_VALU per launch (profiles/)"}
    wpmc = pmc_per_launch("waveform", a.n, TAPS, a.precision, kern["waveform"]["templates_per_launch"])
    if "fma_f64" in wpmc:
        tw = kern["waveform"]["avg_ms"] * 1e-3
        kern["waveform"]["fp64_tflops"] = workcount.executed_flops(0, wpmc["fma_f64"]) / tw / 1e12
        kern["waveform"]["fp64_frac"] = kern["waveform"]["fp64_tflops"] / workcount.VALU_PEAK_TFLOPS
        kern["waveform"]["fp32_tflops"] = workcount.executed_flops(wpmc["fma_f32"], 0) / tw / 1e12
        kern["waveform"]["valu_insts_per_cycle_per_cu"] = workcount.issue_rate(wpmc["valu"], tw)
    mixed_err = mixed_vs_fp64(lib, inputs, ctx, g, P, modes, orb, tdi, S, a.coarse) \
        if prec == lib.LT_MIXED else None
    out = {
        "metric": "logL evals/s (1M-sample precessing AET); ESS/s learned vs plain proposal",
        "value": value, "unit": "logL evals/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32" if prec == lib.LT_MIXED else "f64", "data": "synthetic",
        "config": {"workload": "precessing 5-mode PhenomT-form, 2^20 samples at 5 s, Keplerian arms, TDI-2 AET, "
                               "K=%d Lagrange, batch %d uneven lengths" % (TAPS, a.batch),
                   "global_batch": a.batch, "seq_len": a.n, "parallelism": "single GPU",
                   "active_sample_fraction": active_frac,
                   "precision": a.precision, "waveform_grid": "every sample" if a.coarse == 1 else
                   "every second sample, linear in between", "templates_valid": n_ok,
                   "launch_shape": tuning},
        "kernels_ms": kern,
        "roofline": roof,
        "mixed_vs_fp64": mixed_err,
    }
    if a.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = {"read": src.numel() * 4, "write": dst.numel() * 4, "launches": 3}
    ctx.close()
    if not a.no_sampler:
        runs = [("sampler", sampler_bench, {}), ("ess", ess_bench, {"p_flow": a.p_flow})]
        if not a.no_ess_precessing:
            runs.append(("ess_precessing", ess_bench, {"precessing": True, "p_flow": a.p_flow}))
        for key, fn, kw in runs:
            try:
                out[key] = fn(lib, inputs, prec, **kw)
            except Exception as e:                      # reported, the throughput line still prints
                out[key] = {"error": "%s: %s" % (type(e).__name__, e)}
            print("%s done" % key, file=sys.stderr, flush=True)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, P, TAPS)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
