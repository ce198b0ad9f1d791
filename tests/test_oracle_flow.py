"""Pins of the oracle flow (P27): invertibility, log-det, gradients, learning a Gaussian."""
import math

import numpy as np
import pytest

from oracle import flow as fl


def _rand_params(d, L, H, seed):
    P = fl.init_params(d, L, H, seed)
    rng = np.random.default_rng(seed + 1)
    for p in P:                                  # non-trivial, well-conditioned output layer
        p["W3"] = rng.normal(size=p["W3"].shape) * 0.3 / np.sqrt(p["W3"].shape[1])
        p["b3"] = rng.normal(size=p["b3"].shape) * 0.1
        p["b1"] = rng.normal(size=p["b1"].shape) * 0.1
    return P


@pytest.mark.parametrize("d", [11, 14])
def test_inverse_roundtrip(d):
    P = _rand_params(d, 8, 32, 0)
    mu, sig = np.linspace(-1, 1, d), np.linspace(0.5, 2, d)
    x = mu + sig * np.random.default_rng(2).normal(size=(50, d))
    z, lq = fl.forward(P, x, mu, sig)
    x2, lq2 = fl.inverse(P, z, mu, sig)
    assert np.max(np.abs(x2 - x)) < 1e-10
    assert np.max(np.abs(lq2 - lq)) < 1e-10


def test_logdet_against_numerical_jacobian():
    """P27: log q from the couplings equals the brute-force change of variables."""
    d = 6
    P = _rand_params(d, 8, 16, 3)
    mu, sig = np.zeros(d), np.ones(d) * 1.5
    x = np.random.default_rng(4).normal(size=(3, d))
    for xi in x:
        z, lq = fl.forward(P, xi[None], mu, sig)
        J = np.zeros((d, d))
        h = 1e-6
        for k in range(d):
            e = np.zeros(d)
            e[k] = h
            J[:, k] = (fl.forward(P, (xi + e)[None], mu, sig)[0][0] - fl.forward(P, (xi - e)[None], mu, sig)[0][0]) / (2 * h)
        brute = -0.5 * z[0] @ z[0] - 0.5 * d * math.log(2 * math.pi) + np.log(abs(np.linalg.det(J)))
        assert abs(brute - lq[0]) < 1e-6 + 1e-9 * abs(lq[0])


def test_gradients_against_central_differences():
    """P27: manual backpropagation equals central differences of the loss."""
    d = 5
    P = _rand_params(d, 4, 8, 5)
    mu, sig = np.zeros(d), np.ones(d)
    x = np.random.default_rng(6).normal(size=(20, d)) * 1.3
    loss, G = fl.nll_and_grad(P, x, mu, sig)
    rng = np.random.default_rng(7)
    for l in (0, 3):
        for k in ("W1", "b1", "W2", "W3", "b3"):
            idx = tuple(rng.integers(0, s) for s in P[l][k].shape)
            old = P[l][k][idx]
            h = 1e-6
            P[l][k][idx] = old + h
            lp = fl.nll_and_grad(P, x, mu, sig)[0]
            P[l][k][idx] = old - h
            lm = fl.nll_and_grad(P, x, mu, sig)[0]
            P[l][k][idx] = old
            assert abs((lp - lm) / (2 * h) - G[l][k][idx]) < 1e-6 * max(1.0, abs(G[l][k][idx]))


def test_learns_a_gaussian():
    """P27: trained on Gaussian samples the flow recovers the mean and covariance."""
    d = 3
    rng = np.random.default_rng(8)
    A = rng.normal(size=(d, d))
    C = A @ A.T + np.eye(d)
    m = np.array([1.0, -2.0, 3.0])
    x = rng.multivariate_normal(m, C, size=4000)
    mu, sig = x.mean(0), x.std(0)
    P = fl.init_params(d, 4, 32, 9)
    opt = fl.Adam(P, lr=3e-3)
    for it in range(400):
        b = x[rng.integers(0, x.shape[0], 256)]
        _, G = fl.nll_and_grad(P, b, mu, sig)
        opt.step(P, G)
    xs, _ = fl.inverse(P, rng.normal(size=(20000, d)), mu, sig)
    assert np.allclose(xs.mean(0), m, atol=0.15)
    assert np.allclose(np.cov(xs.T), C, atol=0.25 * np.abs(C).max())
    exact = -0.5 * np.einsum("ni,ij,nj->n", x - m, np.linalg.inv(C), x - m) - 0.5 * np.log(np.linalg.det(2 * np.pi * C))
    assert abs(fl.forward(P, x, mu, sig)[1].mean() - exact.mean()) < 0.1


def _chol_case(d, seed):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(d, d))
    C = A @ A.T + 0.1 * np.eye(d)
    return rng.normal(size=d), C, np.linalg.cholesky(C)


def test_whitened_identity_flow_is_the_gaussian():
    """P27: with a zero output layer and Lw = chol(C), q is N(mu, C) (closed form) and the
    inverse map is x = mu + Lw z."""
    from scipy.stats import multivariate_normal
    d = 6
    mu, C, Lw = _chol_case(d, 1)
    P = fl.init_params(d, 4, 16, 0)
    x = np.random.default_rng(2).multivariate_normal(mu, C, size=40)
    _, lq = fl.forward(P, x, mu, Lw)
    assert np.allclose(lq, multivariate_normal(mu, C).logpdf(x), atol=1e-10)
    z = np.random.default_rng(3).normal(size=(40, d))
    xs, lqs = fl.inverse(P, z, mu, Lw)
    assert np.allclose(xs, mu + z @ Lw.T, atol=1e-12)
    assert np.allclose(lqs, multivariate_normal(mu, C).logpdf(xs), atol=1e-10)


def test_diagonal_matrix_equals_vector_sigma():
    d = 5
    P = _rand_params(d, 4, 16, 4)
    mu, sig = np.linspace(-1, 1, d), np.linspace(0.5, 2, d)
    x = mu + sig * np.random.default_rng(5).normal(size=(30, d))
    z1, l1 = fl.forward(P, x, mu, sig)
    z2, l2 = fl.forward(P, x, mu, np.diag(sig))
    assert np.allclose(z1, z2, atol=1e-14) and np.allclose(l1, l2, atol=1e-12)


def test_whitened_roundtrip_and_gradients():
    d = 7
    mu, C, Lw = _chol_case(d, 6)
    P = _rand_params(d, 4, 16, 7)
    x = np.random.default_rng(8).multivariate_normal(mu, C, size=20)
    z, lq = fl.forward(P, x, mu, Lw)
    x2, lq2 = fl.inverse(P, z, mu, Lw)
    assert np.max(np.abs(x2 - x)) < 1e-10 and np.max(np.abs(lq2 - lq)) < 1e-10
    loss, G = fl.nll_and_grad(P, x, mu, Lw)
    assert loss == pytest.approx(-lq.mean(), rel=1e-12)
    h = 1e-6
    for l, k, idx in ((0, "W1", (3, 1)), (2, "b2", (5,)), (3, "W3", (2, 7))):
        old = P[l][k][idx]
        P[l][k][idx] = old + h
        lp = fl.nll_and_grad(P, x, mu, Lw)[0]
        P[l][k][idx] = old - h
        lm = fl.nll_and_grad(P, x, mu, Lw)[0]
        P[l][k][idx] = old
        assert abs((lp - lm) / (2 * h) - G[l][k][idx]) < 1e-6 * max(1.0, abs(G[l][k][idx]))
