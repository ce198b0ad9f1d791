"""The flow in numpy with the library's rounding points: BF16 (round to nearest
even) GEMM operands, FP32 GEMM results, FP64 everywhere else.  Test helper:
it separates what BF16 arithmetic does to the flow (this model against the
FP64 oracle) from what the kernels do (the library against this model).
"""
import numpy as np

from oracle.flow import split, S_MAX, _whiten, _unwhiten


def bf(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _cond(p, u, A):
    uA = bf(u[:, A])
    h1 = bf(np.maximum(f32(uA @ bf(p["W1"]).T + p["b1"]), 0.0))
    h2 = bf(np.maximum(f32(h1 @ bf(p["W2"]).T + p["b2"]), 0.0))
    o = f32(h2 @ bf(p["W3"]).T + p["b3"])
    return uA, h1, h2, o


def forward(P, x, mu, sigma):
    u, lsig = _whiten(x, mu, sigma)
    d = u.shape[1]
    ld = np.zeros(len(u))
    for l, p in enumerate(P):
        A, B = split(d, l)
        o = _cond(p, u, A)[3]
        nb = B.size
        s = S_MAX * np.tanh(o[:, :nb] / S_MAX)
        u = u.copy()
        u[:, B] = u[:, B] * np.exp(s) + o[:, nb:]
        ld += s.sum(1)
    return u, -0.5 * (u * u).sum(1) - 0.5 * d * np.log(2 * np.pi) + ld - lsig


def inverse(P, z, mu, sigma):
    u = np.asarray(z, float).copy()
    d = u.shape[1]
    base = -0.5 * (u * u).sum(1) - 0.5 * d * np.log(2 * np.pi)
    ld = np.zeros(len(u))
    for l in range(len(P) - 1, -1, -1):
        A, B = split(d, l)
        o = _cond(P[l], u, A)[3]
        nb = B.size
        s = S_MAX * np.tanh(o[:, :nb] / S_MAX)
        u[:, B] = (u[:, B] - o[:, nb:]) * np.exp(-s)
        ld += s.sum(1)
    lsig = _whiten(np.zeros((1, d)), np.zeros(d), sigma)[1]
    return _unwhiten(u, mu, sigma), base + ld - lsig


def nll_grad(P, x, mu, sigma):
    u, _ = _whiten(x, mu, sigma)
    n, d = u.shape
    cache = []
    for l, p in enumerate(P):
        A, B = split(d, l)
        uA, h1, h2, o = _cond(p, u, A)
        nb = B.size
        s = S_MAX * np.tanh(o[:, :nb] / S_MAX)
        uB = u[:, B].copy()
        u = u.copy()
        u[:, B] = uB * np.exp(s) + o[:, nb:]
        cache.append((A, B, uA, uB, h1, h2, o, s))
    g_u = u / n
    grads = [None] * len(P)
    for l in range(len(P) - 1, -1, -1):
        A, B, uA, uB, h1, h2, o, s = cache[l]
        p = P[l]
        nb = B.size
        gy = g_u[:, B]
        es = np.exp(s)
        gs = gy * uB * es - 1.0 / n
        go = f32(np.concatenate([gs * (1 - np.tanh(o[:, :nb] / S_MAX) ** 2), gy], 1))
        g = {"W3": bf(go).T @ h2, "b3": go.sum(0)}
        ga2 = f32((bf(go) @ bf(p["W3"])) * (h2 > 0))
        g["W2"], g["b2"] = bf(ga2).T @ h1, ga2.sum(0)
        ga1 = f32((bf(ga2) @ bf(p["W2"])) * (h1 > 0))
        g["W1"], g["b1"] = bf(ga1).T @ uA, ga1.sum(0)
        g_u = g_u.copy()
        g_u[:, B] = gy * es
        g_u[:, A] = g_u[:, A] + bf(ga1) @ bf(p["W1"])
        grads[l] = g
    return grads
