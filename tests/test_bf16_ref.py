"""The BF16 model used by the flow tests rounds to nearest even and stays near the FP64 oracle."""
import numpy as np

import bf16_ref
from oracle import flow as fl


def test_round_to_nearest_even():
    one = 1.0
    ulp = 2.0 ** -7                                 # BF16 spacing in [1, 2)
    x = np.array([one + ulp / 2, one + 1.5 * ulp, one + 0.51 * ulp, -(one + ulp / 2), 3.0e38, 1e-40])
    got = bf16_ref.bf(x)
    assert got[0] == one and got[1] == one + 2 * ulp and got[2] == one + ulp and got[3] == -one
    assert np.isfinite(got[4]) and got[5] >= 0.0


def test_model_close_to_oracle_for_near_identity_layers():
    d, L, H = 14, 8, 256
    P = fl.init_params(d, L, H, 1)
    rng = np.random.default_rng(2)
    for p in P:
        p["W3"] = rng.normal(size=p["W3"].shape) * 0.05 / np.sqrt(H)
        p["b3"] = rng.normal(size=p["b3"].shape) * 0.1
    x = rng.normal(size=(200, d))
    mu, sig = np.zeros(d), np.ones(d)
    e = np.abs(bf16_ref.forward(P, x, mu, sig)[1] - fl.forward(P, x, mu, sig)[1])
    assert np.median(e) < 5e-3 and e.max() < 0.1
    xb, _ = bf16_ref.inverse(P, x, mu, sig)
    xo, _ = fl.inverse(P, x, mu, sig)
    assert np.max(np.abs(xb - xo)) < 0.05
