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

# algorithmic work per template-sample of the dominant kernels (design notes)
N_SAMPLES = 2 ** 20
BATCH = 256
TAPS = 8


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=BATCH)
    ap.add_argument("--n", type=int, default=N_SAMPLES)
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=3)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (known traffic) to calibrate HBM counters")
    return ap.parse_args()


def cpu_baseline(g, params, taps):
    """Times the oracle (as it stands) on a bounded sample of the same workload:
    the full chain (polarisations, six links, TDI 2.0 X, Y, Z, A, E, T) for one
    template on a contiguous slice of the 2^20 grid, plus the rfft and band
    inner products of one full-length 3-channel series; scaled to logL/s."""
    import numpy as np
    from oracle import likelihood as olk
    from oracle.orbits import Orbit
    from oracle.response import Response
    from oracle.waveform import Template
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    n = g["n"]
    slice_len = 1 << 13
    r = Response(Template(params[0]), g["t0"], g["dt"], n, Orbit("kepler"), taps=taps, precessing=True,
                 generation=20)
    idx = np.arange(n - slice_len - 4096, n - 4096)
    t0 = time.perf_counter()
    r.aet(idx)
    t_resp = (time.perf_counter() - t0) * (n / slice_len)
    x = np.random.default_rng(0).standard_normal((3, n))
    S = olk.channel_psds(n, g["dt"], 20)
    t0 = time.perf_counter()
    olk.loglike(x, 0.5 * x, S, g["dt"])
    t_fft = time.perf_counter() - t0
    per = t_resp + t_fft
    return {"value": 1.0 / per, "unit": "logL evals/s", "cores": threads if threads > 0 else 1,
            "kind": "oracle",
            "sample": "oracle on template 0: response+TDI on %d of %d samples (scaled x%.0f) + full-length "
                      "rfft/inner products; %.1f s measured" % (slice_len, n, n / slice_len,
                                                              per * slice_len / n + t_fft)}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only (this build has no multi-GPU path); got --gpus %d" % a.gpus,
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2501_08261_amd import inputs, lib
    dev = "cuda:0"
    prec = lib.LT_MIXED if a.precision == "mixed" else lib.LT_FP64
    rdt = lib.real_dtype(prec)
    g = inputs.grid(a.n, 5.0)
    ctx = lib.Context(0)
    modes = ((2, 2), (2, 1), (3, 3), (3, 2), (4, 4))
    cfg = ctx.wf_cfg(modes, True, precision=prec)
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

    # per-kernel averages from HIP events recorded on the launch stream
    ctx.profile_enable(True)
    for _ in range(a.profile_steps):
        step()
    torch.cuda.synchronize()
    ms, cnt = ctx.profile_read(5)
    ctx.profile_enable(False)
    names = ["setup", "tdi_response", "fft_pass1", "fft_pass2_band", "finalize"]
    kern = {names[i]: {"avg_ms": ms[i] / max(cnt[i], 1), "launches": cnt[i]} for i in range(5)}
    n_ok = int((status == 0).sum().item())
    # roofline of the dominant kernel (algorithmic work per template-sample, design notes)
    rsz = 4 if prec == lib.LT_MIXED else 8
    fft_bytes = {"fft_pass1": 3 * 2 * rsz, "fft_pass2_band": 3 * rsz}      # per real sample, per template
    dom = max(kern, key=lambda k: kern[k]["avg_ms"])
    if dom in fft_bytes:
        achieved = fft_bytes[dom] * a.n * a.batch / (kern[dom]["avg_ms"] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": 8000.0, "unit": "GB/s", "frac": achieved / 8000.0,
                "traffic": None, "kernel": dom}
    else:
        from paper_2501_08261_amd import workcount
        flops = workcount.tdi_flops_per_sample(TAPS, 20, precessing=True, modes=len(modes))
        achieved = flops * a.n * a.batch / (kern[dom]["avg_ms"] * 1e-3) / 1e12
        peak = 78.6 if prec == lib.LT_FP64 else 157.3
        roof = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": None, "kernel": dom}
    out = {
        "metric": "logL evals/s (1M-sample precessing AET)",
        "value": value, "unit": "logL evals/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32" if prec == lib.LT_MIXED else "f64", "data": "synthetic",
        "config": {"workload": "precessing 5-mode PhenomT-form, 2^20 samples at 5 s, Keplerian arms, TDI-2 AET, "
                               "K=%d Lagrange, batch %d uneven lengths" % (TAPS, a.batch),
                   "global_batch": a.batch, "seq_len": a.n, "parallelism": "single GPU",
                   "precision": a.precision, "templates_valid": n_ok},
        "kernels_ms": kern,
        "roofline": roof,
    }
    if a.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = {"read": src.numel() * 4, "write": dst.numel() * 4, "launches": 3}
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, P, TAPS)
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
