"""The comparison runs of the paper's Tabs. II-III through the library (Fisher widths only, the
MCMC replay is `python -m paper_2501_08261_amd.studies`): the higher modes narrow the distance
and inclination (they break the iota-D degeneracy of the (2,2) mode, Sec. III), one channel
constrains less than two, and the T channel adds little at low frequency."""
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_fisher_widths_across_configurations():
    from paper_2501_08261_amd import inputs, lib, studies
    runs = {r[0]: r for r in studies.RUNS}
    out = {}
    for label in ("T-AET", "THM-AET", "THM-A", "THM-AE"):
        _, modes, ch, gen, orb = runs[label]
        out[label] = studies.run_one(lib, inputs, label, modes, ch, gen, orb, n=1 << 13, fisher_only=True)
    i_d, i_iota = studies.NAMES10.index("D_L"), studies.NAMES10.index("iota")
    s = {k: v["sigma_fisher"] for k, v in out.items()}
    assert s["THM-AET"][i_d] < 0.5 * s["T-AET"][i_d]
    assert s["THM-AET"][i_iota] < 0.5 * s["T-AET"][i_iota]
    assert all(a >= b for a, b in zip(s["THM-A"], s["THM-AE"]))
    assert all(abs(a / b - 1.0) < 0.2 for a, b in zip(s["THM-AE"], s["THM-AET"]))
    assert out["THM-A"]["snr"] < out["THM-AE"]["snr"] <= out["THM-AET"]["snr"]
