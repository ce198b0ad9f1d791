"""lt_tdi_loglike_noalloc (the library's fixed scratch, for callers that cannot allocate) against
lt_tdi_loglike on the same inputs: bit-identical logL, logL_full and status on two calls in a
row, the second with fewer templates and a shorter grid (the scratch keeps the first call's
contents), in both precisions; a grid too large for the scratch and a grid with no FFT plan in
the context are refused before any launch."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle.waveform import MODES_ALL
from paper_2501_08261_amd import inputs

DEV = "cuda:0"


def _case(lib, ctx, n, B, seed, precision):
    g = inputs.grid(n, 5.0)
    P = inputs.draw_templates(seed, B, g, precessing=True, before_end=1000.0)
    P[1, 4] = 1.5                                    # unphysical: status 1, logL = -inf
    cfg, orb, tdi = ctx.wf_cfg(MODES_ALL, True, precision=precision), ctx.orbit("kepler"), ctx.tdi_cfg(20, 7, 8)
    S = torch.zeros((3, n // 2 + 1), dtype=torch.float64, device=DEV)
    lib.psd_sangria(g, 20, S)
    d = torch.zeros((1, 3, n), dtype=lib.real_dtype(precision), device=DEV)
    ctx.lisa_tdi_response(torch.as_tensor(P[:1], device=DEV), g, cfg, orb, tdi, d)
    dd = torch.zeros(1, dtype=torch.float64, device=DEV)
    ctx.noise_inner(d, g, S, dd, precision=precision)
    torch.cuda.synchronize()
    return g, torch.as_tensor(P, device=DEV), cfg, orb, tdi, S, d[0], float(dd.item())


def _outs(B):
    return (torch.full((B,), 7.0, dtype=torch.float64, device=DEV), torch.full((B,), 7.0, dtype=torch.float64, device=DEV),
            torch.full((B,), -7, dtype=torch.int32, device=DEV))


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_matches_loglike(precision):
    from paper_2501_08261_amd import lib
    ctx = lib.Context(0)
    for n, B, seed in ((2 ** 18, 21, 71), (2 ** 16, 5, 72)):     # second call: smaller input
        g, P, cfg, orb, tdi, S, d, dd = _case(lib, ctx, n, B, seed, precision)
        full_b, one_b = ctx.workspace_size(B, g, cfg, tdi)
        print("n %d batch %d: one template needs %d bytes, the whole batch %d" % (n, B, one_b, full_b), flush=True)
        ref = _outs(B)
        ctx.tdi_loglike(P, g, cfg, orb, tdi, S, d, dd, *ref)        # also builds the plan and the node table
        got = _outs(B)
        ctx.tdi_loglike_noalloc(P, g, cfg, orb, tdi, S, d, dd, *got)
        torch.cuda.synchronize()
        for a, b in zip(ref, got):
            assert torch.equal(a, b), (n, B)
        st = got[2].cpu().numpy()
        assert st[1] == 1 and np.all(np.delete(st, 1) == 0)
        assert got[1][0].item() == 0.0                               # template 0 is the data
    ctx.close()


def test_noalloc_refusals():
    from paper_2501_08261_amd import lib
    ctx = lib.Context(0)
    # FP64 at 2^21 samples: one template needs more than the fixed scratch
    n = 2 ** 21
    g = inputs.grid(n, 5.0)
    cfg, orb, tdi = ctx.wf_cfg(MODES_ALL, True), ctx.orbit("kepler"), ctx.tdi_cfg(20, 7, 8)
    P = torch.as_tensor(inputs.draw_templates(3, 1, g, precessing=True), device=DEV)
    S = torch.zeros((3, n // 2 + 1), dtype=torch.float64, device=DEV)
    d = torch.zeros((3, n), dtype=torch.float64, device=DEV)
    lo = torch.zeros(1, dtype=torch.float64, device=DEV)
    with pytest.raises(lib.LisaTDError, match="scratch"):
        ctx.tdi_loglike_noalloc(P, g, cfg, orb, tdi, S, d, 0.0, lo)
    # a grid whose FFT plan this fresh context has not built
    n = 6000
    g = inputs.grid(n, 5.0)
    S = torch.zeros((3, n // 2 + 1), dtype=torch.float64, device=DEV)
    d = torch.zeros((3, n), dtype=torch.float64, device=DEV)
    with pytest.raises(lib.LisaTDError, match="plan"):
        ctx.tdi_loglike_noalloc(P, g, cfg, orb, tdi, S, d, 0.0, lo)
    torch.cuda.synchronize()
    ctx.close()
