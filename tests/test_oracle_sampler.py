"""Pins of the oracle sampler: Philox known answers, Gaussian moments, tempering, ESS."""
import math
import os

import numpy as np
import pytest

from oracle.sampler import PTSampler, philox4x32_10, gaussian_logl, integrated_time

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def test_philox_known_answers():
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(x, 16) for x in line.split()]
        got = philox4x32_10(np.array([v[:4]], dtype=np.uint64), (v[4], v[5]))[0]
        assert [int(x) for x in got] == v[6:]


def test_gaussian_moments():
    """P26: the T = 1 chain reproduces the mean and covariance of a Gaussian."""
    rng = np.random.default_rng(0)
    d = 3
    A = rng.normal(size=(d, d))
    C = A @ A.T + d * np.eye(d)
    mu = np.array([1.0, -2.0, 0.5])
    s = PTSampler(gaussian_logl(mu, np.linalg.inv(C)), [-50] * d, [50] * d, 32, 1, d, seed=7)
    s.set_state(mu + rng.normal(size=(1, 32, d)))
    chain = []
    for i in range(3000):
        s.step()
        if i >= 500:
            chain.append(s.X[0].copy())
    chain = np.array(chain)
    flat = chain.reshape(-1, d)
    tau = integrated_time(chain).max()
    n_eff = flat.shape[0] / tau
    err = np.sqrt(np.diag(C) / n_eff)
    assert np.all(np.abs(flat.mean(0) - mu) < 5 * err)
    assert np.allclose(np.cov(flat.T), C, rtol=0.2, atol=0.2 * np.sqrt(np.outer(np.diag(C), np.diag(C))).max())
    assert 0.2 < s.acc / s.prop < 0.9


def test_tempering_reaches_both_modes():
    """P26: a separated bimodal target needs the tempering swaps."""
    d = 2
    means = np.array([[-4.0, 0.0], [4.0, 0.0]])
    f = gaussian_logl(means, np.eye(d) * 4.0)
    start = np.tile(means[0], (6, 16, 1)) + 0.1 * np.random.default_rng(1).normal(size=(6, 16, d))
    s = PTSampler(f, [-20, -20], [20, 20], 16, 6, d, seed=3, t_max=200.0)
    s.set_state(start)
    frac = []
    for i in range(1500):
        s.step()
        if i > 300:
            frac.append(np.mean(s.X[0, :, 0] > 0))
    assert 0.3 < np.mean(frac) < 0.7
    assert s.sacc > 0
    cold = PTSampler(f, [-20, -20], [20, 20], 16, 1, d, seed=3)
    cold.set_state(start[:1])
    for _ in range(300):
        cold.step()
    assert np.mean(cold.X[0, :, 0] > 0) < 0.2


def test_integrated_time_ar1():
    """P26: the ESS estimator recovers tau = (1 + rho) / (1 - rho) for AR(1)."""
    rng = np.random.default_rng(5)
    rho, n, w = 0.9, 20000, 8
    x = np.zeros((n, w, 1))
    e = rng.normal(size=(n, w))
    for t in range(1, n):
        x[t, :, 0] = rho * x[t - 1, :, 0] + e[t]
    tau = integrated_time(x)[0]
    assert abs(tau / ((1 + rho) / (1 - rho)) - 1) < 0.1


def _identity_flow(d, L=2, H=8):
    from oracle import flow as fl
    return fl.init_params(d, L, H, 0)           # zero output layer: the identity map


def test_flow_normals_are_standard():
    """P28: the Box-Muller base samples of the flow move are standard normal and uncorrelated."""
    s = PTSampler(lambda x: np.zeros(len(x)), [-1] * 6, [1] * 6, 64, 1, 6, seed=11)
    z = np.concatenate([s.flow_normals(k) for k in range(200)])
    assert np.all(np.abs(z.mean(0)) < 4 / np.sqrt(len(z)))
    assert np.allclose(np.cov(z.T), np.eye(6), atol=0.03)
    assert np.allclose((z ** 4).mean(0), 3.0, atol=0.15)


def test_flow_move_exact_proposal_always_accepted():
    """P28: when q equals the target, the independence move accepts every proposal."""
    d = 4
    m = np.array([1.0, -2.0, 0.5, 3.0])
    sd = np.array([0.5, 2.0, 1.0, 0.1])
    s = PTSampler(gaussian_logl(m, np.diag(1 / sd ** 2)), m - 100, m + 100, 16, 1, d, seed=5)
    s.set_state(m + sd * np.random.default_rng(0).normal(size=(1, 16, d)))
    s.set_flow(_identity_flow(d), m, sd)
    for _ in range(20):
        s.step()
    assert s.fprop == 20 * 16 and s.facc == s.fprop


def test_flow_move_keeps_the_target():
    """P28: with a mismatched flow the chain still samples the target (the q(x)/q(y) correction)."""
    rng = np.random.default_rng(3)
    d = 2
    C = np.array([[1.0, 0.6], [0.6, 2.0]])
    m = np.array([0.5, -1.0])
    s = PTSampler(gaussian_logl(m, np.linalg.inv(C)), [-40] * d, [40] * d, 32, 1, d, seed=9)
    s.set_state(m + rng.multivariate_normal(np.zeros(d), C, size=(1, 32)))
    s.set_flow(_identity_flow(d), m + np.array([1.0, -1.0]), np.array([2.0, 2.5]))
    chain = []
    for i in range(2500):
        s.step()
        if i >= 200:
            chain.append(s.X[0].copy())
    chain = np.array(chain)
    flat = chain.reshape(-1, d)
    tau = integrated_time(chain).max()
    err = np.sqrt(np.diag(C) / (flat.shape[0] / tau))
    assert np.all(np.abs(flat.mean(0) - m) < 5 * err)
    assert np.allclose(np.cov(flat.T), C, atol=0.15)
    assert 0.1 < s.facc / s.fprop < 0.9


def test_flow_move_lowers_autocorrelation():
    """P28: a proposal close to the target decorrelates the cold chain faster than stretch moves alone."""
    rng = np.random.default_rng(4)
    d = 3
    A = rng.normal(size=(d, d))
    C = A @ A.T + 0.1 * np.eye(d)
    m = np.zeros(d)
    f = gaussian_logl(m, np.linalg.inv(C))
    taus = []
    for use_flow in (False, True):
        s = PTSampler(f, [-60] * d, [60] * d, 16, 1, d, seed=2)
        s.set_state(rng.multivariate_normal(m, C, size=(1, 16)))
        if use_flow:
            s.set_flow(_identity_flow(d), m, np.sqrt(np.diag(C)) * 1.2)
        chain = []
        for i in range(1500):
            s.step()
            chain.append(s.X[0].copy())
        taus.append(integrated_time(np.array(chain)).max())
    assert taus[1] < 0.7 * taus[0]


def test_package_autocorr_time_matches_oracle():
    """The package's host ESS estimator agrees with the oracle's on AR(1) chains."""
    from paper_2501_08261_amd.diagnostics import autocorr_time
    rng = np.random.default_rng(6)
    n, w = 5000, 6
    x = np.zeros((n, w, 2))
    e = rng.normal(size=(n, w, 2))
    rhos = np.array([0.5, 0.95])
    for t in range(1, n):
        x[t] = rhos * x[t - 1] + e[t]
    assert np.allclose(autocorr_time(x), integrated_time(x), rtol=1e-9)


def _fold_target(m0, s0, P, c0, lo0, hi0, with_copies):
    """log density in x0 of N(fold(x0); m0, s0) on [lo0, hi0], fold into [c0, c0 + P);
    with_copies: divided by the number of copies of fold(x0) in the range (then it equals
    the density the folded flow move proposes, copies chosen uniformly)."""
    def f(x):
        v = c0 + ((x[:, 0] - c0) - P * np.floor((x[:, 0] - c0) / P))
        out = -0.5 * ((v - m0) / s0) ** 2 - 0.5 * x[:, 1] ** 2
        if with_copies:
            n = np.floor((hi0 - v) / P) - np.ceil((lo0 - v) / P) + 1
            out = out - np.log(n)
        return out
    return f


def test_flow_fold_exact_proposal_always_accepted():
    """P29: with the fold, a flow equal to the folded target accepts every proposal inside the
    window and rejects the rest (the copy count differs across the range: a move that dropped
    the -ln n terms would reject some)."""
    P, c0, lo0, hi0 = 2.0, -1.0, -2.0, 1.5
    m, sd = np.array([0.2, 0.0]), np.array([0.4, 1.0])
    s = PTSampler(_fold_target(m[0], sd[0], P, c0, lo0, hi0, True), [lo0, -50], [hi0, 50], 16, 1, 2, seed=21)
    rng = np.random.default_rng(1)
    s.set_state(np.stack([rng.uniform(-0.9, 0.9, 16), rng.normal(size=16)], 1)[None])
    s.set_flow(_identity_flow(2), m, sd)
    s.set_flow_fold(0, P, c0)
    expect = 0
    for _ in range(20):
        yf = m[0] + sd[0] * s.flow_normals(s.step_count)[:, 0]
        expect += int(np.sum((yf >= c0) & (yf < c0 + P)))
        s.step()
    assert s.fprop == 320 and 0 < s.fprop - expect
    assert s.facc == expect


def test_flow_fold_keeps_the_target():
    """P29: with the fold and a mismatched flow, the chain spreads over the copies of the
    symmetric target with the target's masses (two modes 5 sd apart: the stretch moves alone
    rarely cross)."""
    from scipy.stats import norm
    P, c0, lo0, hi0 = 2.0, -1.0, -2.0, 1.5
    m0, s0 = 0.2, 0.4
    s = PTSampler(_fold_target(m0, s0, P, c0, lo0, hi0, False), [lo0, -50], [hi0, 50], 32, 1, 2, seed=23)
    rng = np.random.default_rng(2)
    s.set_state(np.stack([m0 + s0 * rng.normal(size=32), rng.normal(size=32)], 1)[None])
    s.set_flow(_identity_flow(2), np.array([0.0, 0.5]), np.array([0.6, 1.5]))
    s.set_flow_fold(0, P, c0)
    chain = []
    for i in range(3000):
        s.step()
        if i >= 200:
            chain.append(s.X[0, :, 0].copy())
    x = np.array(chain)
    cdf = lambda a, b: norm.cdf(b, m0, s0) - norm.cdf(a, m0, s0)
    mass = np.array([cdf(0.0, 1.0), cdf(-1.0, 1.0), cdf(-1.0, -0.5)])     # x0 in [-2,-1), [-1,1), [1,1.5]
    mass /= mass.sum()
    frac = np.array([np.mean(x < -1.0), np.mean((x >= -1.0) & (x < 1.0)), np.mean(x >= 1.0)])
    tau = integrated_time(x[:, :, None]).max()
    err = np.sqrt(mass * (1 - mass) / (x.size / tau))
    assert np.all(np.abs(frac - mass) < 5 * err + 1e-3), (frac, mass)
    assert 0.2 < s.facc / s.fprop < 0.95


def _curved_flow(d, seed=7, scale=0.25):
    """A nonlinear flow: random output layers, so the Jacobian varies over the space."""
    from oracle import flow as fl
    P = fl.init_params(d, 4, 16, seed)
    rng = np.random.default_rng(seed + 1)
    for p in P:
        p["W3"] = rng.normal(size=p["W3"].shape) * scale / np.sqrt(p["W3"].shape[1])
        p["b3"] = rng.normal(size=p["b3"].shape) * 0.1
    return P


def test_flow_walk_keeps_the_target():
    """P30: the latent random walk through a curved flow samples the target: the acceptance
    carries the ratio of the flow's Jacobians, log q - log N at both ends (dropping the log N
    terms, or the Jacobians, biases the moments below by many standard errors)."""
    rng = np.random.default_rng(8)
    d = 2
    C = np.array([[1.0, 0.5], [0.5, 1.5]])
    m = np.array([0.3, -0.7])
    s = PTSampler(gaussian_logl(m, np.linalg.inv(C)), [-40] * d, [40] * d, 32, 1, d, seed=31)
    s.set_state(m + rng.multivariate_normal(np.zeros(d), C, size=(1, 32)))
    s.set_flow(_curved_flow(d), m + np.array([0.5, 0.2]), np.array([1.3, 0.9]))
    s.set_flow_walk(0.9)
    chain = []
    for i in range(3000):
        s.step()
        if i >= 200:
            chain.append(s.X[0].copy())
    chain = np.array(chain)
    flat = chain.reshape(-1, d)
    tau = integrated_time(chain).max()
    err = np.sqrt(np.diag(C) / (flat.shape[0] / tau))
    assert np.all(np.abs(flat.mean(0) - m) < 5 * err)
    assert np.allclose(np.cov(flat.T), C, atol=0.12)
    assert 0.2 < s.facc / s.fprop < 0.95


def test_flow_mix_keeps_the_target():
    """P36: the flow move mixed with the stretch move at rate p_flow (a Philox draw per step
    decides): the chain still samples the target with a mismatched flow, the flow move runs on
    the expected fraction of steps, and p_flow = 0 is the plain sampler, draw for draw."""
    rng = np.random.default_rng(5)
    d = 2
    C = np.array([[1.0, -0.4], [-0.4, 0.5]])
    m = np.array([-0.3, 0.8])
    start = m + rng.multivariate_normal(np.zeros(d), C, size=(1, 32))
    s = PTSampler(gaussian_logl(m, np.linalg.inv(C)), [-40] * d, [40] * d, 32, 1, d, seed=21)
    s.set_state(start)
    s.set_flow(_identity_flow(d), m + np.array([-0.8, 0.6]), np.array([1.5, 1.2]))
    s.set_flow_mix(0.3)
    chain = []
    n = 3000
    for i in range(n):
        s.step()
        if i >= 200:
            chain.append(s.X[0].copy())
    chain = np.array(chain)
    flat = chain.reshape(-1, d)
    tau = integrated_time(chain).max()
    err = np.sqrt(np.diag(C) / (flat.shape[0] / tau))
    assert np.all(np.abs(flat.mean(0) - m) < 5 * err)
    assert np.allclose(np.cov(flat.T), C, atol=0.1)
    assert abs(s.flow_steps / n - 0.3) < 4 * math.sqrt(0.3 * 0.7 / n)
    assert s.fprop == 32 * s.flow_steps and 0 < s.facc < s.fprop
    # p_flow = 0: identical to the sampler without a flow
    a = PTSampler(gaussian_logl(m, np.linalg.inv(C)), [-40] * d, [40] * d, 32, 1, d, seed=22)
    b = PTSampler(gaussian_logl(m, np.linalg.inv(C)), [-40] * d, [40] * d, 32, 1, d, seed=22)
    a.set_state(start)
    b.set_state(start)
    b.set_flow(_identity_flow(d), m, np.ones(d))
    b.set_flow_mix(0.0)
    for _ in range(50):
        a.step()
        b.step()
    assert np.array_equal(a.X, b.X) and b.fprop == 0


def test_flow_exclusive_keeps_the_target():
    """P37: on the steps that run the flow move, the flow move replaces the cold rung's stretch
    moves (the hotter rungs keep theirs): the cold chain still samples the target with a
    mismatched flow, and exactly the cold rows of the flow steps go unproposed."""
    rng = np.random.default_rng(6)
    d, W, T = 2, 32, 2
    C = np.array([[1.0, 0.5], [0.5, 0.8]])
    m = np.array([0.4, -0.6])
    start = m + rng.multivariate_normal(np.zeros(d), C, size=(T, W))
    s = PTSampler(gaussian_logl(m, np.linalg.inv(C)), [-40] * d, [40] * d, W, T, d, seed=23, t_max=4.0)
    s.set_state(start)
    s.set_flow(_identity_flow(d), m + np.array([0.7, -0.5]), np.array([1.4, 1.3]))
    s.set_flow_mix(0.5)
    s.set_flow_exclusive(True)
    chain = []
    n = 3000
    for i in range(n):
        s.step()
        if i >= 200:
            chain.append(s.X[0].copy())
    chain = np.array(chain)
    flat = chain.reshape(-1, d)
    tau = integrated_time(chain).max()
    err = np.sqrt(np.diag(C) / (flat.shape[0] / tau))
    assert np.all(np.abs(flat.mean(0) - m) < 5 * err)
    assert np.allclose(np.cov(flat.T), C, atol=0.1)
    assert abs(s.flow_steps / n - 0.5) < 4 * math.sqrt(0.25 / n)
    assert s.prop == n * T * W - s.flow_steps * W
    assert s.fprop == W * s.flow_steps and 0 < s.facc < s.fprop


def _two_mode_run(monkeypatch=None, plant=False, mixture=True, n=2500, seed=31):
    d, W = 2, 32
    m = np.array([[-6.0, 0.5], [6.0, -0.5]])
    icov = np.eye(d)
    rng = np.random.default_rng(seed)
    start = m[0] + rng.normal(size=(1, W, d))          # every walker starts in mode 1
    s = PTSampler(gaussian_logl(m, icov), [-40] * d, [40] * d, W, 1, d, seed=seed)
    s.set_state(start)
    s.set_flow(_identity_flow(d), m[0] + 0.2, np.array([1.3, 1.2]))
    if mixture:
        s.set_flow_mixture(_identity_flow(d), m[1] - 0.1, np.array([1.2, 1.4]), 0.4)
    if plant:
        # a plausible mistake: the proposal density of the component that was drawn only
        monkeypatch.setattr(PTSampler, "_mix_logq", lambda self, x: flow_forward(self.flow, x))
    chain = []
    for i in range(n):
        s.step()
        if i >= 300:
            chain.append(s.X[0].copy())
    return np.array(chain), m, s


def flow_forward(fl_tuple, x):
    from oracle import flow as fl
    P, mu, sigma = fl_tuple
    return fl.forward(P, x, mu, sigma)[1]


def test_flow_mixture_keeps_the_target(monkeypatch):
    """P38: a mixture of two flows, one on each mode of a two-mode Gaussian, as the independence
    proposal (q = w1 q1 + w2 q2, the component drawn per walker): from a start in one mode the
    chain holds both modes with their equal weights and the target's moments; one flow alone
    does not reach the second mode; using the drawn component's density instead of the mixture's
    biases the weights."""
    chain, m, s = _two_mode_run()
    flat = chain.reshape(-1, 2)
    frac2 = np.mean(flat[:, 0] > 0)
    assert abs(frac2 - 0.5) < 0.05
    for k, sel in ((0, flat[:, 0] < 0), (1, flat[:, 0] > 0)):
        assert np.all(np.abs(flat[sel].mean(0) - m[k]) < 0.08)
        assert np.allclose(np.cov(flat[sel].T), np.eye(2), atol=0.12)
    assert 0.3 < s.facc / s.fprop < 0.95
    one, _, _ = _two_mode_run(mixture=False, n=800)
    assert np.mean(one.reshape(-1, 2)[:, 0] > 0) < 0.02
    bad, _, _ = _two_mode_run(monkeypatch, plant=True)
    assert abs(np.mean(bad.reshape(-1, 2)[:, 0] > 0) - 0.5) > 0.1
