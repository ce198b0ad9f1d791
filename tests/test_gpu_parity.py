"""GPU (HIP C-ABI) versus the FP64 oracle, element by element.

Tolerance metric (per template and channel): max_n |g_n - o_n| / max_n |o_n|;
T, a cancellation channel (X + Y + Z ~ 0 for equal arms), is measured against
the largest channel of its template.
FP64 mode: waveform and TDI samples <= 1e-9.  logL: 1e-6 absolute plus
1e-11 (d|d): two FP64 evaluations of a ~1e4 rad phase differ by ~1e-12 of h,
which bounds every inner product at that relative level.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import likelihood as olk
from oracle.orbits import Orbit as OOrbit
from oracle.response import Response
from oracle.twist import polarizations as opol
from oracle.waveform import Template, cp_modes, MODES_ALL
from paper_2501_08261_amd import inputs

DEV = "cuda:0"


@pytest.fixture(scope="module")
def lt():
    from paper_2501_08261_amd import lib
    ctx = lib.Context(0)
    yield lib, ctx
    torch.cuda.synchronize()
    ctx.close()


def relerr(g, o):
    g, o = np.asarray(g), np.asarray(o)
    return np.max(np.abs(g - o)) / max(np.max(np.abs(o)), 1e-300)


def _dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def _aligned_batch(seed, B, g):
    return inputs.draw_templates(seed, B, g, precessing=False, before_end=1000.0)


@pytest.mark.parametrize("n", [4096, 5000])
def test_modes_parity(lt, n):
    lib, ctx = lt
    g = inputs.grid(n, 5.0)
    P = _aligned_batch(11, 6, g)
    P[0] = inputs.single_template_case()[1]
    P[0, 11] = inputs.peak_time(g, 1000.0)
    out = torch.zeros((P.shape[0], 5, n, 2), dtype=torch.float64, device=DEV)
    ctx.phenomt_modes(_dev(P), g, ctx.wf_cfg(MODES_ALL), out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    t = g["t0"] + np.arange(n) * g["dt"]
    for b in range(P.shape[0]):
        want = cp_modes(Template(P[b]), t, MODES_ALL)
        for i in range(5):
            gm = got[b, i, :, 0] + 1j * got[b, i, :, 1]
            assert relerr(gm, want[i]) < 1e-9, (b, i)


@pytest.mark.parametrize("precessing", [False, True])
def test_polarization_parity(lt, precessing):
    lib, ctx = lt
    n = 6000
    g = inputs.grid(n, 5.0)
    P = inputs.draw_templates(5 + precessing, 8, g, precessing=precessing, before_end=1000.0)
    out = torch.zeros((P.shape[0], 2, n), dtype=torch.float64, device=DEV)
    ctx.phenomt_polarizations(_dev(P), g, ctx.wf_cfg(MODES_ALL, precessing), out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    t = g["t0"] + np.arange(n) * g["dt"]
    for b in range(P.shape[0]):
        hp, hc = opol(Template(P[b]), t, MODES_ALL, precessing)
        assert relerr(got[b, 0], hp) < 1e-9 and relerr(got[b, 1], hc) < 1e-9, b


def _assert_aet(got, want, tol, tag=None):
    scale = np.max(np.abs(want))
    for c in range(3):
        norm = max(np.max(np.abs(want[c])), scale if c == 2 else 0.0)
        assert np.max(np.abs(got[c] - want[c])) < tol * norm, (tag, c)


def _oracle_aet(p, g, orbit, taps, modes, precessing, gen, xyz=False):
    r = Response(Template(p), g["t0"], g["dt"], g["n"], OOrbit(orbit), taps=taps, modes=modes,
                 precessing=precessing, generation=gen)
    r.cache_full_grid()
    idx = np.arange(g["n"])
    return np.array(r.xyz(idx) if xyz else r.aet(idx))


@pytest.mark.parametrize("precessing,n", [(False, 6001), (True, 5998)])
def test_polarization_parity_coarse(lt, precessing, n):
    """N2: the waveform on every second sample, the mean of the neighbours in between, against
    the oracle's definition (odd and even grid lengths: the last odd sample needs the waveform
    one step past the grid)."""
    lib, ctx = lt
    g = inputs.grid(n, 5.0)
    P = inputs.draw_templates(7 + precessing, 6, g, precessing=precessing, before_end=1000.0)
    out = torch.zeros((P.shape[0], 2, n), dtype=torch.float64, device=DEV)
    ctx.phenomt_polarizations(_dev(P), g, ctx.wf_cfg(MODES_ALL, precessing, coarse=2), out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for b in range(P.shape[0]):
        r = Response(Template(P[b]), g["t0"], g["dt"], n, OOrbit("static"), modes=MODES_ALL, precessing=precessing,
                     coarse=2)
        hp, hc = r.h_grid(np.arange(n))
        assert relerr(got[b, 0], hp) < 1e-9 and relerr(got[b, 1], hc) < 1e-9, b


def test_tdi_parity_coarse(lt):
    """N2: response and TDI from the coarse-grid waveform (FP64) against the oracle."""
    lib, ctx = lt
    n = 5000
    g = inputs.grid(n, 5.0)
    P = inputs.draw_templates(55, 3, g, precessing=True, before_end=1000.0)
    out = torch.zeros((P.shape[0], 3, n), dtype=torch.float64, device=DEV)
    ctx.lisa_tdi_response(_dev(P), g, ctx.wf_cfg(MODES_ALL, True, coarse=2), ctx.orbit("kepler"),
                          ctx.tdi_cfg(20, 7, 8), out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for b in range(P.shape[0]):
        r = Response(Template(P[b]), g["t0"], g["dt"], n, OOrbit("kepler"), taps=8, modes=MODES_ALL,
                     precessing=True, generation=20, coarse=2)
        r.cache_full_grid()
        _assert_aet(got[b], np.array(r.aet(np.arange(n))), 1e-9, b)


@pytest.mark.parametrize("orbit,gen,taps,precessing", [
    ("static", 15, 2, False), ("static", 15, 8, False), ("kepler", 20, 2, False),
    ("kepler", 20, 8, True), ("kepler", 20, 32, True), ("static", 20, 4, True), ("kepler", 15, 6, False)])
def test_tdi_parity(lt, orbit, gen, taps, precessing):
    lib, ctx = lt
    n = 5000                                    # ragged last tile
    g = inputs.grid(n, 5.0)
    P = inputs.draw_templates(100 + taps, 3, g, precessing=precessing, before_end=1000.0)
    out = torch.zeros((P.shape[0], 3, n), dtype=torch.float64, device=DEV)
    st = torch.full((P.shape[0],), -7, dtype=torch.int32, device=DEV)
    ctx.lisa_tdi_response(_dev(P), g, ctx.wf_cfg(MODES_ALL, precessing), ctx.orbit(orbit),
                          ctx.tdi_cfg(gen, 7, taps), out, st)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert np.all(st.cpu().numpy() == 0)
    for b in range(P.shape[0]):
        want = _oracle_aet(P[b], g, orbit, taps, MODES_ALL, precessing, gen)
        _assert_aet(got[b], want, 1e-9, b)


@pytest.mark.parametrize("gen,taps,precessing", [(20, 8, True), (15, 2, False)])
def test_tdi_parity_orbit_table(lt, gen, taps, precessing):
    """N4: an orbit file (hourly positions and light times, Keplerian ellipses sampled by the
    input generator) read through the table orbit kind: FP64 response against the oracle on
    the same table, and close to the analytic Kepler orbit it samples (the table's
    interpolation moves positions by ~1 mm and light times by < 1e-11 s)."""
    lib, ctx = lt
    n = 5000                                    # ragged last tile
    g = inputs.grid(n, 5.0)
    tab = inputs.orbit_table(-86400.0, 3600.0, 60)
    P = inputs.draw_templates(300 + taps, 3, g, precessing=precessing, before_end=1000.0)
    outs = []
    for orb in (ctx.orbit("table", table=tab), ctx.orbit("kepler")):
        out = torch.zeros((P.shape[0], 3, n), dtype=torch.float64, device=DEV)
        st = torch.full((P.shape[0],), -7, dtype=torch.int32, device=DEV)
        ctx.lisa_tdi_response(_dev(P), g, ctx.wf_cfg(MODES_ALL, precessing), orb, ctx.tdi_cfg(gen, 7, taps), out, st)
        torch.cuda.synchronize()
        assert np.all(st.cpu().numpy() == 0)
        outs.append(out.cpu().numpy())
    for b in range(P.shape[0]):
        r = Response(Template(P[b]), g["t0"], g["dt"], n, OOrbit("table", table=tab), taps=taps, modes=MODES_ALL,
                     precessing=precessing, generation=gen)
        r.cache_full_grid()
        want = np.array(r.aet(np.arange(n)))
        _assert_aet(outs[0][b], want, 1e-9, b)
        _assert_aet(outs[0][b], outs[1][b], 1e-6, b)
    short = inputs.orbit_table(-86400.0, 3600.0, 20)          # ends before the grid does
    with pytest.raises(lib.LisaTDError):
        ctx.lisa_tdi_response(_dev(P), g, ctx.wf_cfg(MODES_ALL, precessing), ctx.orbit("table", table=short),
                              ctx.tdi_cfg(gen, 7, taps), torch.zeros((P.shape[0], 3, n), dtype=torch.float64,
                                                                     device=DEV))


# Mixed precision (FP32 response and TDI, FP64 times and delays): the output
# error is set by FP32 rounding of h, which y = h(t_s) - h(t_r) turns into an
# absolute error of order u max|h| (u = 2^-24) whatever the size of y, and
# which the K-tap interpolations and the TDI sums accumulate.  Measured over
# 15 templates (M = 1.7e5 - 8.2e6, K = 2 - 16, both generations, both orbit
# kinds) the error per channel was C u max|h| with C between 3 and 42; the
# bound below is 24 sqrt(K) u max|h|, at least 1.6 times every measurement,
# in the metric of R20 (relative to the channel's maximum).
U32 = 2.0 ** -24


@pytest.mark.parametrize("orbit,gen,taps,precessing,dt", [
    ("kepler", 20, 8, True, 5.0), ("kepler", 20, 2, False, 5.0), ("kepler", 15, 8, False, 5.0),
    ("static", 20, 8, True, 5.0), ("kepler", 20, 16, True, 5.0), ("kepler", 20, 8, True, 1.0),
    ("kepler", 20, 24, False, 5.0), ("kepler", 20, 32, True, 5.0)])
def test_tdi_parity_mixed(lt, orbit, gen, taps, precessing, dt):
    """Mixed path against the oracle: combined per-link filters (K <= 16 at dt = 5 s), per-term
    Taylor weights (dt = 1 s, where the filters would exceed their length bound) and direct
    FP32 weights (K > 16)."""
    lib, ctx = lt
    n = 5000
    g = inputs.grid(n, dt)
    P = inputs.draw_templates(100 + taps, 3, g, precessing=precessing, before_end=1000.0)
    out = torch.zeros((P.shape[0], 3, n), dtype=torch.float32, device=DEV)
    st = torch.full((P.shape[0],), -7, dtype=torch.int32, device=DEV)
    ctx.lisa_tdi_response(_dev(P), g, ctx.wf_cfg(MODES_ALL, precessing, precision=lib.LT_MIXED),
                          ctx.orbit(orbit), ctx.tdi_cfg(gen, 7, taps), out, st)
    torch.cuda.synchronize()
    got = out.double().cpu().numpy()
    assert np.all(st.cpu().numpy() == 0)
    for b in range(P.shape[0]):
        r = Response(Template(P[b]), g["t0"], g["dt"], n, OOrbit(orbit), taps=taps, modes=MODES_ALL,
                     precessing=precessing, generation=gen)
        r.cache_full_grid()
        idx = np.arange(n)
        want = np.array(r.aet(idx))
        hp, hc = r.h_grid(idx)
        hmax = max(np.max(np.abs(hp)), np.max(np.abs(hc)))
        scale = np.max(np.abs(want))
        for c in range(3):
            norm = max(np.max(np.abs(want[c])), scale if c == 2 else 0.0)
            err = np.max(np.abs(got[b, c] - want[c]))
            assert err < 24.0 * math.sqrt(taps) * U32 * hmax, (b, c, err / (U32 * hmax), err / norm)


@pytest.mark.parametrize("precision", [0, 1])
def test_tdi_full_size_sampled(lt, precision):
    """The bench workload at full size (256 precessing templates, 2^20 samples, Kepler arms,
    TDI 2.0, K = 8, one launch): the lightest, a median and the heaviest template checked
    against the oracle at sampled outputs
    (every sample of the last 2400, where the merger and each channel's maximum lie, and 200
    drawn over the rest)."""
    lib, ctx = lt
    n, B, K = 2 ** 20, 256, 8
    g = inputs.grid(n, 5.0)
    P = inputs.draw_templates(3, B, g, precessing=True)
    rdt = lib.real_dtype(precision)
    out = torch.zeros((B, 3, n), dtype=rdt, device=DEV)
    st = torch.full((B,), -7, dtype=torch.int32, device=DEV)
    ctx.lisa_tdi_response(_dev(P), g, ctx.wf_cfg(MODES_ALL, True, precision=precision), ctx.orbit("kepler"),
                          ctx.tdi_cfg(20, 7, K), out, st)
    torch.cuda.synchronize()
    assert np.all(st.cpu().numpy() == 0)
    rng = np.random.default_rng(7)
    idx = np.unique(np.concatenate([np.arange(n - 2400, n), rng.integers(0, n - 2400, 200)]))
    M = P[:, 0] + P[:, 1]
    for b in (int(np.argmin(M)), int(np.argsort(M)[B // 2]), int(np.argmax(M))):
        got = out[b][:, torch.as_tensor(idx, device=DEV)].double().cpu().numpy()
        r = Response(Template(P[b]), g["t0"], g["dt"], n, OOrbit("kepler"), taps=K, modes=MODES_ALL,
                     precessing=True, generation=20)
        want = np.array(r.aet(idx))
        if precision == 0:
            # both sides round the absolute sample time (up to n dt) to u64 n samples;
            # heavy templates' TDI 2.0 channels are (2 pi f L)^2 below h, so that floor
            # is measured against max|h| (the highest mode frequency is below 2 omega_ring)
            tpl = Template(P[b])
            hp, hc = r.h_grid(np.arange(n - 2400, n))
            hmax = max(np.max(np.abs(hp)), np.max(np.abs(hc)))
            floor = 32.0 * 2.0 ** -53 * n * min(2.0 * (tpl.w_lo + tpl.Delta) * g["dt"], math.pi) * hmax
            scale = np.max(np.abs(want))
            for c in range(3):
                norm = max(np.max(np.abs(want[c])), scale if c == 2 else 0.0)
                assert np.max(np.abs(got[c] - want[c])) < 1e-9 * norm + floor, (b, c)
        else:
            hp, hc = r.h_grid(np.arange(n - 2400, n))
            hmax = max(np.max(np.abs(hp)), np.max(np.abs(hc)))
            assert np.max(np.abs(got - want)) < 24.0 * math.sqrt(K) * U32 * hmax, b


def test_loglike_full_size_composition(lt):
    """The bench workload at full size in its launch configuration (256 precessing templates,
    2^20 samples, Kepler arms, TDI 2.0, K = 8, mixed precision, one launch per kernel): a
    template equal to the data has logL_full exactly 0 and logL = dd / 2; for the lightest, a
    median and the heaviest template, logL_full equals -1/2 (r|r) of the residual r = h - d
    built from the response (checked against the oracle at this size in
    test_tdi_full_size_sampled) and the band inner product (checked against the oracle at
    2^20 in test_band_inner_parity)."""
    lib, ctx = lt
    n, B, K = 2 ** 20, 256, 8
    g = inputs.grid(n, 5.0)
    P = inputs.draw_templates(3, B, g, precessing=True)
    inj = inputs.tab1_injection(True, g)
    P[17] = inj
    cfg = ctx.wf_cfg(MODES_ALL, True, precision=lib.LT_MIXED)
    orb, tdi = ctx.orbit("kepler"), ctx.tdi_cfg(20, 7, K)
    S = _psd_dev(lib, g, 20)
    d = torch.zeros((1, 3, n), dtype=torch.float32, device=DEV)
    ctx.lisa_tdi_response(_dev(inj[None]), g, cfg, orb, tdi, d)
    dd = torch.zeros(1, dtype=torch.float64, device=DEV)
    ctx.noise_inner(d, g, S, dd, precision=lib.LT_MIXED)
    torch.cuda.synchronize()
    ddv = float(dd.item())
    logl = torch.zeros(B, dtype=torch.float64, device=DEV)
    full = torch.zeros(B, dtype=torch.float64, device=DEV)
    st = torch.full((B,), -7, dtype=torch.int32, device=DEV)
    ctx.tdi_loglike(_dev(P), g, cfg, orb, tdi, S, d[0], ddv, logl, full, st)
    torch.cuda.synchronize()
    assert np.all(st.cpu().numpy() == 0)
    assert full[17].item() == 0.0 and logl[17].item() == 0.5 * ddv
    M = P[:, 0] + P[:, 1]
    pick = [int(np.argmin(M)), int(np.argsort(M)[B // 2]), int(np.argmax(M))]
    h = torch.zeros((3, 3, n), dtype=torch.float32, device=DEV)
    ctx.lisa_tdi_response(_dev(P[pick]), g, cfg, orb, tdi, h)
    rr = torch.zeros(3, dtype=torch.float64, device=DEV)
    ctx.noise_inner((h - d).contiguous(), g, S, rr, precision=lib.LT_MIXED)
    torch.cuda.synchronize()
    want = -0.5 * rr.cpu().numpy()
    got = full.cpu().numpy()[pick]
    assert np.allclose(got, want, rtol=1e-12, atol=1e-9 * ddv), (got, want)
    assert np.allclose(logl.cpu().numpy()[pick], got + 0.5 * ddv, rtol=1e-12, atol=1e-9 * ddv)


def test_xyz_output(lt):
    lib, ctx = lt
    n = 3000
    g = inputs.grid(n, 5.0)
    P = inputs.draw_templates(3, 2, g, precessing=False, before_end=1000.0)
    out = torch.zeros((2, 3, n), dtype=torch.float64, device=DEV)
    ctx.lisa_tdi_response(_dev(P), g, ctx.wf_cfg(MODES_ALL), ctx.orbit("kepler"),
                          ctx.tdi_cfg(20, 7, 4, out_xyz=True), out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for b in range(2):
        want = _oracle_aet(P[b], g, "kepler", 4, MODES_ALL, False, 20, xyz=True)
        for c in range(3):
            assert relerr(got[b, c], want[c]) < 1e-9


@pytest.mark.parametrize("n", [1000, 17280, 16384, 2 ** 20])
@pytest.mark.parametrize("precision", [0, 1])
def test_rfft_parity(lt, n, precision):
    lib, ctx = lt
    rows = 3
    x = inputs.random_series(n, (rows, n))
    dt = 5.0
    xd = _dev(x, lib.real_dtype(precision))
    out = torch.zeros((rows, n // 2 + 1, 2), dtype=lib.real_dtype(precision), device=DEV)
    ctx.rfft(xd, dt, out, precision)
    torch.cuda.synchronize()
    got = out.cpu().double().numpy()
    got = got[..., 0] + 1j * got[..., 1]
    tol = 1e-13 if precision == 0 else 2e-6
    for r in range(rows):
        want = olk.rfft_dt(x[r], dt)
        assert relerr(got[r], want) < tol, r


def _psd_dev(lib, g, gen):
    S = torch.zeros((3, g["n"] // 2 + 1), dtype=torch.float64, device=DEV)
    lib.psd_sangria(g, gen, S)
    return S


@pytest.mark.parametrize("gen", [15, 20])
def test_psd_parity(lt, gen):
    lib, ctx = lt
    g = inputs.grid(17280, 5.0)
    S = _psd_dev(lib, g, gen).cpu().numpy()
    want = olk.channel_psds(g["n"], g["dt"], gen)
    assert np.all(np.isinf(S[:, 0]))
    assert np.max(np.abs(S[:, 1:] / want[:, 1:] - 1)) < 1e-12


def test_single_template_loglike(lt):
    """One-day (2,2) case, static arms, TDI 1.5, K = 2 and 8, FP64: logL within 1e-6."""
    lib, ctx = lt
    g, inj, tmpl = inputs.single_template_case()
    S = _psd_dev(lib, g, 15)
    Snp = olk.channel_psds(g["n"], g["dt"], 15)
    for taps in (2, 8):
        cfg = ctx.wf_cfg(((2, 2),))
        orb, tdi = ctx.orbit("static"), ctx.tdi_cfg(15, 7, taps)
        d = torch.zeros((1, 3, g["n"]), dtype=torch.float64, device=DEV)
        ctx.lisa_tdi_response(_dev(inj[None]), g, cfg, orb, tdi, d)
        dd = torch.zeros(1, dtype=torch.float64, device=DEV)
        ctx.noise_inner(d, g, S, dd)
        logl = torch.zeros(2, dtype=torch.float64, device=DEV)
        full = torch.zeros(2, dtype=torch.float64, device=DEV)
        st = torch.zeros(2, dtype=torch.int32, device=DEV)
        ctx.tdi_loglike(_dev(np.stack([inj, tmpl])), g, cfg, orb, tdi, S, d[0], float(dd.item()), logl, full, st)
        torch.cuda.synchronize()
        od = _oracle_aet(inj, g, "static", taps, ((2, 2),), False, 15)
        oh = _oracle_aet(tmpl, g, "static", taps, ((2, 2),), False, 15)
        want_dd = olk.noise_inner(od, Snp, g["dt"])
        tol = 1e-6 + 1e-11 * want_dd
        assert abs(dd.item() - want_dd) < 1e-11 * want_dd
        l0, f0 = olk.loglike(od, od, Snp, g["dt"])
        l1, f1 = olk.loglike(od, oh, Snp, g["dt"])
        gl, gf = logl.cpu().numpy(), full.cpu().numpy()
        assert gf[0] == 0.0 and f0 == 0.0            # h = d exactly on both sides
        assert abs(gl[0] - l0) < tol
        assert abs(gl[1] - l1) < tol and abs(gf[1] - f1) < tol
        assert np.all(st.cpu().numpy() == 0)


def test_noisy_data_loglike(lt):
    """N3: Gaussian noise drawn from the PSD added to the injection (one-day case, static arms,
    TDI 1.5, K = 8, FP64): logL and logL_full of the injection and a template against the
    oracle on the same noisy data, and logL_full at the injection equals -(n|n)/2."""
    lib, ctx = lt
    g, inj, tmpl = inputs.single_template_case()
    S = _psd_dev(lib, g, 15)
    Snp = olk.channel_psds(g["n"], g["dt"], 15)
    noise = inputs.colored_noise(31, S.cpu().numpy(), g["dt"])
    cfg = ctx.wf_cfg(((2, 2),))
    orb, tdi = ctx.orbit("static"), ctx.tdi_cfg(15, 7, 8)
    h = torch.zeros((1, 3, g["n"]), dtype=torch.float64, device=DEV)
    ctx.lisa_tdi_response(_dev(inj[None]), g, cfg, orb, tdi, h)
    nz = _dev(noise[None])
    d = h + nz
    dd = torch.zeros(1, dtype=torch.float64, device=DEV)
    nn = torch.zeros(1, dtype=torch.float64, device=DEV)
    ctx.noise_inner(d, g, S, dd)
    ctx.noise_inner(nz, g, S, nn)
    logl = torch.zeros(2, dtype=torch.float64, device=DEV)
    full = torch.zeros(2, dtype=torch.float64, device=DEV)
    st = torch.zeros(2, dtype=torch.int32, device=DEV)
    ctx.tdi_loglike(_dev(np.stack([inj, tmpl])), g, cfg, orb, tdi, S, d[0], float(dd.item()), logl, full, st)
    torch.cuda.synchronize()
    od = _oracle_aet(inj, g, "static", 8, ((2, 2),), False, 15)
    oh = _oracle_aet(tmpl, g, "static", 8, ((2, 2),), False, 15)
    dn = od + noise
    want_dd = olk.noise_inner(dn, Snp, g["dt"])
    want_nn = olk.noise_inner(noise, Snp, g["dt"])
    tol = 1e-6 + 1e-11 * want_dd
    assert abs(dd.item() - want_dd) < 1e-11 * want_dd
    assert abs(nn.item() - want_nn) < 1e-11 * want_nn
    gl, gf = logl.cpu().numpy(), full.cpu().numpy()
    for j, oo in enumerate((od, oh)):
        l, f = olk.loglike(dn, oo, Snp, g["dt"])
        assert abs(gl[j] - l) < tol and abs(gf[j] - f) < tol, j
    assert abs(gf[0] + 0.5 * nn.item()) < 1e-6 + 1e-11 * nn.item()
    assert np.all(st.cpu().numpy() == 0)


@pytest.mark.parametrize("precision", [0, 1])
def test_loglike_chunks_equal_split_calls(lt, precision):
    """Batches above 256 templates run in chunks of 256: bit-identical to the same templates
    split over smaller calls, and one invalid template stays isolated to its own slot."""
    lib, ctx = lt
    n = 8192
    g = inputs.grid(n, 5.0)
    B = 300
    P = inputs.draw_templates(21, B, g, precessing=True, before_end=1000.0)
    P[77, 4] = 1.5                                  # |chi1| > 1: status 1, logL = -inf
    S = _psd_dev(lib, g, 20)
    cfg, orb, tdi = ctx.wf_cfg(MODES_ALL, True, precision=precision), ctx.orbit("kepler"), ctx.tdi_cfg(20, 7, 8)
    d = torch.zeros((1, 3, n), dtype=lib.real_dtype(precision), device=DEV)
    ctx.lisa_tdi_response(_dev(P[:1]), g, cfg, orb, tdi, d)
    dd = torch.zeros(1, dtype=torch.float64, device=DEV)
    ctx.noise_inner(d, g, S, dd, precision=precision)
    torch.cuda.synchronize()
    Pd = _dev(P)
    one = torch.zeros(B, dtype=torch.float64, device=DEV)
    one_full = torch.zeros(B, dtype=torch.float64, device=DEV)
    st1 = torch.full((B,), -7, dtype=torch.int32, device=DEV)
    ctx.tdi_loglike(Pd, g, cfg, orb, tdi, S, d[0], float(dd.item()), one, one_full, st1)
    two = torch.zeros(B, dtype=torch.float64, device=DEV)
    two_full = torch.zeros(B, dtype=torch.float64, device=DEV)
    st2 = torch.full((B,), -7, dtype=torch.int32, device=DEV)
    for a, b in ((0, 100), (100, 130), (130, B)):   # chunk boundaries elsewhere
        ctx.tdi_loglike(Pd[a:b].contiguous(), g, cfg, orb, tdi, S, d[0], float(dd.item()), two[a:b], two_full[a:b],
                        st2[a:b])
    torch.cuda.synchronize()
    assert torch.equal(one, two) and torch.equal(one_full, two_full) and torch.equal(st1, st2)
    s1 = st1.cpu().numpy()
    assert s1[77] == 1 and np.all(np.delete(s1, 77) == 0)
    assert np.isneginf(one[77].item()) and np.all(np.isfinite(np.delete(one.cpu().numpy(), 77)))
    assert one_full[0].item() == 0.0                # template 0 is the data


def test_loglike_mixed_close(lt):
    """Mixed precision on the one-day case (static arms, TDI 1.5, K = 8): logL of the injection
    and of two nearby templates against the oracle on the same FP32 data.  The residual form
    -(r|r)/2 turns an error e of the GPU's FP32 residual into -(r|e) - (e|e)/2, so the logL
    error is bounded by |e| |r| + |e|^2 / 2 with |e| the measured error of the GPU's own FP32
    response (factor 2 of margin), plus u log2(n) (r|r) for the FP32 FFT of r and 1e-3."""
    lib, ctx = lt
    g, inj, tmpl = inputs.single_template_case()
    S = _psd_dev(lib, g, 15)
    Snp = olk.channel_psds(g["n"], g["dt"], 15)
    orb, tdi = ctx.orbit("static"), ctx.tdi_cfg(15, 7, 8)
    cfg32 = ctx.wf_cfg(((2, 2),), precision=lib.LT_MIXED)
    P = np.stack([inj, inj, inj])
    P[1, 0] *= 1.0 + 1e-6
    P[2, 12] += 1e-3
    H = [_oracle_aet(p, g, "static", 8, ((2, 2),), False, 15) for p in P]
    d32 = H[0].astype(np.float32).astype(np.float64)
    dd = olk.noise_inner(d32, Snp, g["dt"])
    logl = torch.zeros(3, dtype=torch.float64, device=DEV)
    full = torch.zeros(3, dtype=torch.float64, device=DEV)
    ctx.tdi_loglike(_dev(P), g, cfg32, orb, tdi, S, _dev(d32, torch.float32), dd, logl, full)
    out = torch.zeros((3, 3, g["n"]), dtype=torch.float32, device=DEV)
    ctx.lisa_tdi_response(_dev(P), g, cfg32, orb, tdi, out)
    torch.cuda.synchronize()
    gl, gf, hg = logl.cpu().numpy(), full.cpu().numpy(), out.double().cpu().numpy()
    for j in range(3):
        l, f = olk.loglike(d32, H[j], Snp, g["dt"])
        e = math.sqrt(olk.noise_inner(hg[j] - H[j], Snp, g["dt"]))
        rn = math.sqrt(max(-2.0 * f, 0.0))
        bound = 2.0 * (e * rn + 0.5 * e * e) + U32 * math.log2(g["n"]) * rn * rn + 1e-3
        assert e < 2e-6 * math.sqrt(dd), j
        assert abs(gl[j] - l) < bound and abs(gf[j] - f) < bound, (j, gl[j] - l, bound)


def test_invalid_template_status(lt):
    lib, ctx = lt
    g = inputs.grid(4096, 5.0)
    P = _aligned_batch(1, 2, g)
    P[1, 4] = 1.5                                  # |chi1| >= 1
    S = _psd_dev(lib, g, 15)
    d = torch.zeros((1, 3, g["n"]), dtype=torch.float64, device=DEV)
    logl = torch.zeros(2, dtype=torch.float64, device=DEV)
    st = torch.zeros(2, dtype=torch.int32, device=DEV)
    ctx.tdi_loglike(_dev(P), g, ctx.wf_cfg(), ctx.orbit(), ctx.tdi_cfg(), S, d[0], 0.0, logl, status=st)
    torch.cuda.synchronize()
    assert st.cpu().tolist() == [0, 1]
    assert np.isfinite(logl[0].item()) and logl[1].item() == -math.inf


def test_host_errors(lt):
    lib, ctx = lt
    g = inputs.grid(4096, 5.0)
    P = _dev(_aligned_batch(1, 1, g))
    out = torch.zeros((1, 3, 4096), dtype=torch.float64, device=DEV)
    with pytest.raises(lib.LisaTDError):
        ctx.lisa_tdi_response(P, g, ctx.wf_cfg(), ctx.orbit(), ctx.tdi_cfg(taps=3), out)
    with pytest.raises(lib.LisaTDError):
        ctx.lisa_tdi_response(P, g, ctx.wf_cfg(), ctx.orbit(), ctx.tdi_cfg(generation=17), out)
    with pytest.raises(lib.LisaTDError):
        ctx.rfft(torch.zeros((1, 14), dtype=torch.float64, device=DEV), 5.0,
                 torch.zeros((1, 8, 2), dtype=torch.float64, device=DEV))


@pytest.mark.parametrize("n", [17280, 2 ** 20])
@pytest.mark.parametrize("precision", [0, 1])
def test_band_inner_parity(lt, n, precision):
    """sum_c (x_c|x_c) over the band: FFT passes plus the fused weighted reduction."""
    lib, ctx = lt
    g = inputs.grid(n, 5.0)
    x = inputs.random_series(n + precision, (2, 3, n), 1e-20)
    S = _psd_dev(lib, g, 20)
    out = torch.zeros(2, dtype=torch.float64, device=DEV)
    ctx.noise_inner(_dev(x, lib.real_dtype(precision)), g, S, out, precision=precision)
    torch.cuda.synchronize()
    Snp = olk.channel_psds(n, g["dt"], 20)
    xs = x.astype(np.float32).astype(np.float64) if precision else x
    for b in range(2):
        want = olk.noise_inner(xs[b], Snp, g["dt"])
        assert abs(out[b].item() - want) < (1e-12 if precision == 0 else 1e-5) * want
