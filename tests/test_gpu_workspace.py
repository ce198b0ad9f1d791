"""lt_tdi_loglike with a caller-provided workspace (lt_workspace_size): bit-identical to the
context's own scratch for a full-size workspace and for one that holds only a few templates
per chunk; a workspace below one template's needs is refused before any launch."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle.waveform import MODES_ALL
from paper_2501_08261_amd import inputs

DEV = "cuda:0"


@pytest.mark.parametrize("precision", [0, 1])
def test_workspace_matches_context_scratch(precision):
    from paper_2501_08261_amd import lib
    ctx = lib.Context(0)
    n, B = 8192, 37
    g = inputs.grid(n, 5.0)
    P = inputs.draw_templates(61, B, g, precessing=True, before_end=1000.0)
    P[5, 4] = 1.5                                   # unphysical: status 1 in every layout
    cfg, orb, tdi = ctx.wf_cfg(MODES_ALL, True, precision=precision), ctx.orbit("kepler"), ctx.tdi_cfg(20, 7, 8)
    S = torch.zeros((3, n // 2 + 1), dtype=torch.float64, device=DEV)
    lib.psd_sangria(g, 20, S)
    d = torch.zeros((1, 3, n), dtype=lib.real_dtype(precision), device=DEV)
    ctx.lisa_tdi_response(torch.as_tensor(P[:1], device=DEV), g, cfg, orb, tdi, d)
    dd = torch.zeros(1, dtype=torch.float64, device=DEV)
    ctx.noise_inner(d, g, S, dd, precision=precision)
    torch.cuda.synchronize()
    Pd = torch.as_tensor(P, device=DEV)
    full_b, one_b = ctx.workspace_size(B, g, cfg, tdi)
    assert 0 < one_b < full_b

    def run(ws):
        lo = torch.zeros(B, dtype=torch.float64, device=DEV)
        fu = torch.zeros(B, dtype=torch.float64, device=DEV)
        st = torch.full((B,), -7, dtype=torch.int32, device=DEV)
        ctx.tdi_loglike(Pd, g, cfg, orb, tdi, S, d[0], float(dd.item()), lo, fu, st, workspace=ws)
        torch.cuda.synchronize()
        return lo, fu, st

    ref = run(None)
    for nbytes in (full_b, one_b + (full_b - one_b) // 10, one_b):   # chunks of 37, a few, and 1
        ws = torch.full((nbytes,), 0xA5, dtype=torch.uint8, device=DEV)   # stale contents must not matter
        got = run(ws)
        for a, b in zip(ref, got):
            assert torch.equal(a, b), nbytes
    s = ref[2].cpu().numpy()
    assert s[5] == 1 and np.all(np.delete(s, 5) == 0)
    assert ref[1][0].item() == 0.0
    with pytest.raises(lib.LisaTDError, match="workspace"):
        run(torch.zeros(one_b - 256, dtype=torch.uint8, device=DEV))
    ctx.close()
