"""Batch-means effective sample size and quantile errors of ensemble chains, against closed
forms: independent samples, AR(1) walkers (tau = (1 + rho) / (1 - rho)), and walkers that share
a common AR(1) component, which the per-walker autocorrelation time does not see."""
import math

import numpy as np

from paper_2501_08261_amd.diagnostics import autocorr_time, batch_ess, batch_quantile_se


def _ar1(rng, n, shape, rho):
    x = np.zeros((n,) + shape)
    e = rng.normal(size=(n,) + shape) * math.sqrt(1.0 - rho * rho)
    x[0] = rng.normal(size=shape)
    for t in range(1, n):
        x[t] = rho * x[t - 1] + e[t]
    return x


def test_batch_ess_independent_samples():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(4000, 32, 6))
    e = batch_ess(x, n_batches=100)
    assert np.all(np.abs(e / x[..., 0].size - 1.0) < 0.45)
    assert abs(np.median(e) / x[..., 0].size - 1.0) < 0.2


def test_batch_ess_ar1_walkers():
    rng = np.random.default_rng(2)
    rho = 0.8
    x = _ar1(rng, 20000, (8, 3), rho)
    tau = (1 + rho) / (1 - rho)
    e = batch_ess(x, n_batches=50)
    assert np.all(np.abs(e / (x[..., 0].size / tau) - 1.0) < 0.4)


def test_batch_ess_sees_a_shared_component():
    # x[t, w] = c[t] + e[t, w]: c an AR(1) shared by all walkers, e white, unit variances.
    # Ensemble mean of a batch of L steps: var ~ tau_c / L + 1 / (L W), so
    # ESS = steps * 2 / (tau_c + 1 / W), far below steps * W / tau_walker.
    rng = np.random.default_rng(3)
    n, W, rho = 40000, 64, 0.9
    c = _ar1(rng, n, (1, 2), rho)
    x = c + rng.normal(size=(n, W, 2))
    tau_c = (1 + rho) / (1 - rho)
    expect = n * 2.0 / (tau_c + 1.0 / W)
    e = batch_ess(x, n_batches=40)
    assert np.all(np.abs(e / expect - 1.0) < 0.4)
    e_tau = n * W / autocorr_time(x)
    assert np.all(e_tau > 20 * e)


def test_batch_quantile_se_of_independent_normals():
    # the median of N standard normals has standard error sqrt(pi / 2) / sqrt(N)
    rng = np.random.default_rng(4)
    x = rng.normal(size=(2000, 16, 4))
    q, se = batch_quantile_se(x, qs=(0.5,), n_batches=50)
    assert np.all(np.abs(q) < 5 * se)
    expect = math.sqrt(math.pi / 2.0 / x[..., 0].size)
    assert np.all(np.abs(se / expect - 1.0) < 0.45)
