"""Launch shapes of the likelihood (lt_tuning: templates per launch, the response kernel's
work order, one workgroup per item or a persistent grid) change no result: A, E, T and logL
are bit-identical over every shape, in both precisions, on uneven template lengths with an
unphysical template and a ragged last tile; the autotuner picks one of them, caches it by
workload and reads it back."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle.waveform import MODES_ALL
from paper_2501_08261_amd import inputs

DEV = "cuda:0"
SHAPES = [dict(chunk=c, rotate=r, persistent=p, wg_per_cu=w)
          for c in (256, 7, 16) for r in (1, 0) for p, w in ((0, 4), (1, 4), (1, 1), (1, 8))]


def _setup(lib, ctx, n, B, precision):
    g = inputs.grid(n, 5.0)
    P = inputs.draw_templates(91, B, g, precessing=True, before_end=1000.0)
    P[3, 0] = -1.0                                  # unphysical: status 1
    cfg, orb, tdi = ctx.wf_cfg(MODES_ALL, True, precision=precision), ctx.orbit("kepler"), ctx.tdi_cfg(20, 7, 8)
    S = torch.zeros((3, n // 2 + 1), dtype=torch.float64, device=DEV)
    lib.psd_sangria(g, 20, S)
    d = torch.zeros((1, 3, n), dtype=lib.real_dtype(precision), device=DEV)
    ctx.lisa_tdi_response(torch.as_tensor(P[:1], device=DEV), g, cfg, orb, tdi, d)
    dd = torch.zeros(1, dtype=torch.float64, device=DEV)
    ctx.noise_inner(d, g, S, dd, precision=precision)
    torch.cuda.synchronize()
    return g, torch.as_tensor(P, device=DEV), cfg, orb, tdi, S, d[0], float(dd.item())


@pytest.mark.parametrize("precision", [0, 1])
def test_launch_shapes_are_bit_identical(precision):
    from paper_2501_08261_amd import lib
    ctx = lib.Context(0)
    n, B = 10000, 37
    g, P, cfg, orb, tdi, S, d, dd = _setup(lib, ctx, n, B, precision)
    ref = None
    for shape in SHAPES:
        ctx.set_tuning(**shape)
        lo = torch.zeros(B, dtype=torch.float64, device=DEV)
        fu = torch.zeros(B, dtype=torch.float64, device=DEV)
        st = torch.full((B,), -7, dtype=torch.int32, device=DEV)
        ctx.tdi_loglike(P, g, cfg, orb, tdi, S, d, dd, lo, fu, st)
        aet = torch.zeros((B, 3, n), dtype=lib.real_dtype(precision), device=DEV)
        ctx.lisa_tdi_response(P, g, cfg, orb, tdi, aet)
        torch.cuda.synchronize()
        got = (lo, fu, st, aet)
        if ref is None:
            ref = got
            s = st.cpu().numpy()
            assert s[3] == 1 and np.all(np.delete(s, 3) == 0)
            continue
        for a, b in zip(ref, got):
            assert torch.equal(a, b), shape
    ctx.set_tuning()
    assert ctx.get_tuning() == dict(chunk=256, rotate=1, persistent=0, wg_per_cu=4)
    ctx.close()


def test_autotune_caches_by_workload(tmp_path):
    from paper_2501_08261_amd import lib
    ctx = lib.Context(0)
    n, B = 16384, 150
    g, P, cfg, orb, tdi, S, d, dd = _setup(lib, ctx, n, B, 1)
    path = str(tmp_path / "tuning.txt")
    best, ms = ctx.autotune(P, g, cfg, orb, tdi, S, d, dd, cache_path=path, reps=2)
    assert ms > 0 and best in [dict(chunk=c, rotate=r, persistent=p, wg_per_cu=w) for c in (256, 64, 128)
                               for r in (1, 0) for p, w in ((0, 4), (1, 4), (1, 8))]
    assert ctx.get_tuning() == best
    lines = open(path).read().splitlines()
    assert len(lines) == 1 and "n=16384" in lines[0] and "batch=150" in lines[0]
    ctx.set_tuning()
    again, ms2 = ctx.autotune(P, g, cfg, orb, tdi, S, d, dd, cache_path=path, reps=2)
    assert again == best and ms2 == -1.0
    with pytest.raises(lib.LisaTDError):
        ctx.set_tuning(chunk=0)
    ctx.close()
