"""RealNVP-style normalising flow in numpy FP64.  Test infrastructure only.

The learned proposal is not in the paper (Sec. II.A mentions machine learning
only as a motivation for a Python implementation); its definition here is the
reference of the GPU flow kernels:

* coordinates are whitened, u = Lw^-1 (x - mu), with Lw either the diagonal
  diag(sigma) (sigma a vector) or a lower-triangular matrix with a positive
  diagonal (sigma a matrix, e.g. the Cholesky factor of a sample covariance);
* L affine coupling layers; layer l splits u into a conditioning part A and a
  transformed part B (even l: A = first floor(d/2) coordinates, B = the rest;
  odd l: A = last floor(d/2) coordinates, B = the first d - floor(d/2));
* conditioner MLP: h1 = relu(W1 u_A + b1), h2 = relu(W2 h1 + b2),
  o = W3 h2 + b3 (width H), s = S tanh(o[:d_B] / S) with S = 3, t = o[d_B:];
* y_B = u_B exp(s) + t, y_A = u_A, log|det| += sum(s);
* base density standard normal: log q(x) = -|z|^2/2 - d/2 log(2 pi)
  + sum_l sum(s_l) - sum log diag(Lw);
* training: mean negative log-likelihood of samples, Adam (beta1 0.9,
  beta2 0.999, eps 1e-8).
"""
import math

import numpy as np
from scipy.linalg import solve_triangular

S_MAX = 3.0


def split(d, l):
    da = d // 2
    if l % 2 == 0:
        return np.arange(0, da), np.arange(da, d)
    return np.arange(d - da, d), np.arange(0, d - da)


def init_params(d, n_layers, hidden, seed):
    """He-normal hidden layers from numpy's generator; zero output layer (identity flow)."""
    rng = np.random.default_rng(seed)
    P = []
    for l in range(n_layers):
        A, B = split(d, l)
        P.append({
            "W1": rng.normal(size=(hidden, A.size)) * math.sqrt(2.0 / A.size), "b1": np.zeros(hidden),
            "W2": rng.normal(size=(hidden, hidden)) * math.sqrt(2.0 / hidden), "b2": np.zeros(hidden),
            "W3": np.zeros((2 * B.size, hidden)), "b3": np.zeros(2 * B.size)})
    return P


def _whiten(x, mu, sigma):
    sigma = np.asarray(sigma, float)
    r = np.asarray(x, float) - mu
    if sigma.ndim == 1:
        return r / sigma, np.log(sigma).sum()
    return solve_triangular(sigma, r.T, lower=True).T, np.log(np.diag(sigma)).sum()


def _unwhiten(u, mu, sigma):
    sigma = np.asarray(sigma, float)
    if sigma.ndim == 1:
        return u * sigma + mu
    return u @ sigma.T + mu


def _cond(p, uA):
    a1 = uA @ p["W1"].T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    o = h2 @ p["W3"].T + p["b3"]
    return a1, h1, a2, h2, o


def forward(P, x, mu, sigma):
    """x [n][d] -> z [n][d], log q(x) [n]."""
    u, lsig = _whiten(x, mu, sigma)
    d = u.shape[1]
    ld = np.zeros(u.shape[0])
    for l, p in enumerate(P):
        A, B = split(d, l)
        o = _cond(p, u[:, A])[4]
        nb = B.size
        s = S_MAX * np.tanh(o[:, :nb] / S_MAX)
        u = u.copy()
        u[:, B] = u[:, B] * np.exp(s) + o[:, nb:]
        ld += s.sum(1)
    logq = -0.5 * (u * u).sum(1) - 0.5 * d * math.log(2 * math.pi) + ld - lsig
    return u, logq


def inverse(P, z, mu, sigma):
    """z [n][d] -> x [n][d], log q(x) [n]."""
    u = np.asarray(z, float).copy()
    d = u.shape[1]
    base = -0.5 * (u * u).sum(1) - 0.5 * d * math.log(2 * math.pi)
    ld = np.zeros(u.shape[0])
    for l in range(len(P) - 1, -1, -1):
        p = P[l]
        A, B = split(d, l)
        o = _cond(p, u[:, A])[4]
        nb = B.size
        s = S_MAX * np.tanh(o[:, :nb] / S_MAX)
        u[:, B] = (u[:, B] - o[:, nb:]) * np.exp(-s)
        ld += s.sum(1)
    lsig = _whiten(np.zeros((1, d)), np.zeros(d), sigma)[1]
    return _unwhiten(u, mu, sigma), base + ld - lsig


def nll_and_grad(P, x, mu, sigma):
    """Mean negative log-likelihood of samples x and its gradient (same structure as P)."""
    u, lsig = _whiten(x, mu, sigma)
    n, d = u.shape
    cache = []
    for l, p in enumerate(P):
        A, B = split(d, l)
        uA = u[:, A].copy()
        a1, h1, a2, h2, o = _cond(p, uA)
        nb = B.size
        s = S_MAX * np.tanh(o[:, :nb] / S_MAX)
        uB = u[:, B].copy()
        u = u.copy()
        u[:, B] = uB * np.exp(s) + o[:, nb:]
        cache.append((A, B, uA, uB, a1, h1, a2, h2, o, s))
    logq = -0.5 * (u * u).sum(1) - 0.5 * d * math.log(2 * math.pi) + \
        sum(c[9].sum(1) for c in cache) - lsig
    loss = -logq.mean()
    g_u = u / n                         # d loss / d z
    grads = [None] * len(P)
    for l in range(len(P) - 1, -1, -1):
        A, B, uA, uB, a1, h1, a2, h2, o, s = cache[l]
        p = P[l]
        nb = B.size
        gyB = g_u[:, B]
        es = np.exp(s)
        g_s = gyB * uB * es - 1.0 / n    # from y_B and from -log|det|
        g_t = gyB
        g_uB = gyB * es
        g_oraw = g_s * (1.0 - np.tanh(o[:, :nb] / S_MAX) ** 2)
        g_o = np.concatenate([g_oraw, g_t], axis=1)
        g = {"W3": g_o.T @ h2, "b3": g_o.sum(0)}
        g_h2 = g_o @ p["W3"]
        g_a2 = g_h2 * (a2 > 0)
        g["W2"], g["b2"] = g_a2.T @ h1, g_a2.sum(0)
        g_h1 = g_a2 @ p["W2"]
        g_a1 = g_h1 * (a1 > 0)
        g["W1"], g["b1"] = g_a1.T @ uA, g_a1.sum(0)
        g_uA = g_a1 @ p["W1"]
        g_u = g_u.copy()
        g_u[:, B] = g_uB
        g_u[:, A] = g_u[:, A] + g_uA
        grads[l] = g
    return loss, grads


class Adam:
    def __init__(self, P, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps, self.t = lr, b1, b2, eps, 0
        self.m = [{k: np.zeros_like(v) for k, v in p.items()} for p in P]
        self.v = [{k: np.zeros_like(v) for k, v in p.items()} for p in P]

    def step(self, P, G):
        self.t += 1
        for p, g, m, v in zip(P, G, self.m, self.v):
            for k in p:
                m[k] = self.b1 * m[k] + (1 - self.b1) * g[k]
                v[k] = self.b2 * v[k] + (1 - self.b2) * g[k] ** 2
                mh = m[k] / (1 - self.b1 ** self.t)
                vh = v[k] / (1 - self.b2 ** self.t)
                p[k] = p[k] - self.lr * mh / (np.sqrt(vh) + self.eps)
