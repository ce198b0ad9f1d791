"""The paper's comparison runs (Sec. III, Tabs. II-III) replayed with this library's
PhenomT-form model: for one zero-noise injection, the Fisher widths and the MCMC posterior of
each configuration of

* modes: the (2,2) mode alone against the five modes (the paper's T against THM),
* channels: A against A, E against A, E, T,
* TDI generation: 1.5 against 2.0,
* arms: the static equal-arm triangle against the Keplerian unequal arms (the paper's UA runs
  read ESA orbit files; here the unequal arms are the library's Keplerian orbits),

on the aligned-spin 10-D coordinates (m1, m2, chi1z, chi2z, D_L, iota, phi_ref, beta, lambda,
psi) of the Tab. I aligned injection, a grid of n samples at 5 s ending 2000 s after the merger.
Everything runs through the library (likelihood, Fisher matrix, sampler); numpy only reduces
the chains.

    python -m paper_2501_08261_amd.studies [--n 16384] [--steps 1000] [--fisher-only] > runs.json
"""
import argparse
import json
import math
import sys

import numpy as np

NAMES10 = ["m1", "m2", "chi1z", "chi2z", "D_L", "iota", "phi_ref", "beta", "lambda", "psi"]
FISHER_STEPS_A10 = [1.0, 1.0, 1e-4, 1e-4, 1.0, 1e-5, 1e-5, 1e-5, 1e-5, 1e-5]
MODES_22 = ((2, 2),)
MODES_HM = ((2, 2), (2, 1), (3, 3), (3, 2), (4, 4))

# (label, modes, channels bitmask A=1 E=2 T=4, TDI generation, orbit kind); labels follow the
# paper's tables: T = (2,2) only, THM = higher modes, UA = unequal arms, G2 = TDI 2.0
RUNS = [
    ("T-AET", MODES_22, 7, 15, "static"),
    ("THM-AET", MODES_HM, 7, 15, "static"),
    ("UA-THM-AET", MODES_HM, 7, 15, "kepler"),
    ("THM-A", MODES_HM, 1, 15, "static"),
    ("THM-AE", MODES_HM, 3, 15, "static"),
    ("THM-AET-G2", MODES_HM, 7, 20, "static"),
    ("UA-THM-AET-G2", MODES_HM, 7, 20, "kepler"),
]


def fisher_sigma(G):
    """sqrt(diag(Gamma^-1)), inverted in the basis where Gamma has a unit diagonal (the
    coordinates span many orders of magnitude), eigenvalues floored at 1e-15 of the largest."""
    dg = np.sqrt(np.diag(G))
    ev, V = np.linalg.eigh(G / np.outer(dg, dg))
    ev = np.maximum(ev, 1e-15 * ev.max())
    return np.sqrt(np.diag((V / ev) @ V.T)) / dg


def run_one(lib, inputs, label, modes, channels, generation, orbit_kind, n=1 << 14, W=512, T=8, burn=1000,
            steps=1000, seed=7, fisher_only=False, precision=None, fisher_reg=1e-6):
    import torch
    from paper_2501_08261_amd.diagnostics import autocorr_time
    dev = "cuda:0"
    prec = lib.LT_MIXED if precision is None else precision
    ctx = lib.Context(0)
    g = inputs.grid(n, 5.0)
    cfg = ctx.wf_cfg(modes, False, precision=prec)
    cfg64 = ctx.wf_cfg(modes, False, precision=lib.LT_FP64)
    orb = ctx.orbit(orbit_kind)
    tdi = ctx.tdi_cfg(generation, channels, 8)
    S = torch.zeros((3, n // 2 + 1), dtype=torch.float64, device=dev)
    lib.psd_sangria(g, generation, S)
    inj = inputs.tab1_injection(False, g)
    d = torch.zeros((1, 3, n), dtype=lib.real_dtype(prec), device=dev)
    ctx.lisa_tdi_response(torch.tensor(inj[None], device=dev), g, cfg, orb, tdi, d)
    dd = torch.zeros(1, dtype=torch.float64, device=dev)
    ctx.noise_inner(d, g, S, dd, channels=channels, precision=prec)
    torch.cuda.synchronize()
    x0, lo, hi = inputs.tab1_prior(False, inj)
    G = lib.fisher(ctx, x0, "aligned10", inj[11], FISHER_STEPS_A10, g, cfg64, orb, tdi, S)
    sig_f = fisher_sigma(G)
    out = {"label": label, "modes": len(modes), "channels": "".join(c for c, b in zip("AET", (1, 2, 4))
                                                                    if channels & b),
           "tdi": "2.0" if generation == 20 else "1.5", "arms": "equal (static)" if orbit_kind == "static"
           else "unequal (Kepler)", "snr": math.sqrt(float(dd.item())), "names": NAMES10,
           "sigma_fisher": sig_f.tolist()}
    if fisher_only:
        ctx.close()
        return out
    smp = lib.Sampler(W, T, 10, lo, hi, seed, target="tdi", param_kind="aligned10", t_c=inj[11], g=g, cfg=cfg,
                      orbit=orb, tdi=tdi, psd=S, data_aet=d[0], dd=float(dd.item()))
    smp.set_state(lib.fisher_draw(x0, G, lo, hi, T * W, seed, fisher_reg))
    smp.step(burn)
    chain = []
    for _ in range(steps):
        smp.step(1)
        chain.append(smp.state()[0][0].copy())
    chain = np.array(chain)
    # psi is identified mod pi (h carries exp(2 i psi)): fold around the chain's circular mean
    two = 2.0 * chain[..., 9]
    start = 0.5 * math.atan2(np.sin(two).mean(), np.cos(two).mean()) - 0.5 * math.pi
    chain[..., 9] = start + np.mod(chain[..., 9] - start, math.pi)
    flat = chain.reshape(-1, 10)
    tau = autocorr_time(chain)
    x0f = x0.copy()
    x0f[9] = start + np.mod(x0f[9] - start, math.pi)
    sd = flat.std(0)
    q = np.percentile(flat, [5, 50, 95], axis=0)
    cnt = smp.state()[4]
    smp.close()
    ctx.close()
    out.update({"sigma_mcmc": sd.tolist(), "mcmc_over_fisher": (sd / sig_f).tolist(),
                "median_shift_sigma": ((q[1] - x0f) / sd).tolist(), "q05": q[0].tolist(), "q95": q[2].tolist(),
                "tau_max": float(tau.max()), "ess": float(steps * W / tau.max()),
                "stretch_accept": float(cnt[0] / max(cnt[1], 1)), "swap_accept": float(cnt[2] / max(cnt[3], 1))})
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=1 << 14)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--burn", type=int, default=1000)
    ap.add_argument("--fisher-only", action="store_true")
    ap.add_argument("--only", default=None, help="comma-separated labels")
    a = ap.parse_args(argv)
    from paper_2501_08261_amd import inputs, lib
    res = []
    for label, modes, ch, gen, orb in RUNS:
        if a.only and label not in a.only.split(","):
            continue
        res.append(run_one(lib, inputs, label, modes, ch, gen, orb, n=a.n, burn=a.burn, steps=a.steps,
                           fisher_only=a.fisher_only))
        print("%s done" % label, file=sys.stderr, flush=True)
    print(json.dumps({"n": a.n, "dt": 5.0, "injection": "Tab. I aligned (m1 1e6, m2 7e5 Msun, chi 0.7, 0.4, "
                                                         "D 20 Gpc, iota 149 deg)", "runs": res}))


if __name__ == "__main__":
    main()
