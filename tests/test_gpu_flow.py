"""GPU flow proposal (lt_flow_*) and the sampler's flow move against the oracle.

Tolerances.  The identity flow (zero output layer) is exact in the library's
FP64 coupling path, so it is compared to 1e-12.  A non-trivial flow runs its
conditioner GEMMs on BF16 operands (unit roundoff 2^-9 ~ 2e-3) with FP32
accumulation, and a composition of 8 random layers passes rounding errors on
multiplied by each layer's Lipschitz constant (layers of output scale
0.3 / sqrt(H) make it chaotic in the tails).  Two comparisons therefore:
(1) the library against tests/bf16_ref.py, the same flow in numpy with the
library's rounding points, where only the FP32 summation order differs
(1e-3 on log q, 1 % on gradient blocks); (2) the library against the FP64
oracle, row by row no further than the BF16 model itself is from it (plus
1e-3), for near-identity layers of scale 0.05 / sqrt(H) whose BF16 deviation
stays below about 0.05 on log q and 5 % on gradients.  A wrong GEMM tile
moves log q by about 0.4 and fails both.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import flow as fl
from oracle.sampler import PTSampler, gaussian_logl, integrated_time

import bf16_ref

DEV = "cuda:0"


@pytest.fixture(scope="module")
def lib():
    from paper_2501_08261_amd import lib as L
    return L


def _rand_params(d, L, H, seed, scale=0.05):
    P = fl.init_params(d, L, H, seed)
    rng = np.random.default_rng(seed + 1)
    for p in P:
        p["W3"] = rng.normal(size=p["W3"].shape) * scale / np.sqrt(p["W3"].shape[1])
        p["b3"] = rng.normal(size=p["b3"].shape) * 0.1
        p["b1"] = rng.normal(size=p["b1"].shape) * 0.1
    return P


def _f32(P):
    """The oracle evaluated with the FP32 master weights the library holds."""
    return [{k: np.asarray(v, np.float32).astype(np.float64) for k, v in p.items()} for p in P]


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def test_pack_layout(lib):
    d, L, H = 7, 3, 16
    P = _rand_params(d, L, H, 0)
    f = lib.Flow(d, L, H, 8)
    w = lib.flow_pack(P)
    assert f.num_params == w.size
    f.set_params(w, np.zeros(d), np.ones(d))
    assert np.array_equal(f.get_params(), w)
    Q = lib.flow_unpack(w, d, L, H)
    assert all(np.array_equal(Q[l][k], np.float32(P[l][k])) for l in range(L) for k in P[l])
    f.close()


@pytest.mark.parametrize("n", [1, 37, 300])
def test_identity_flow_is_exact(lib, n):
    d, L, H = 14, 8, 256
    rng = np.random.default_rng(n)
    P = fl.init_params(d, L, H, 3)
    mu, sig = rng.normal(size=d), rng.uniform(0.5, 3.0, size=d)
    f = lib.Flow(d, L, H, 512)
    f.set_params(lib.flow_pack(P), mu, sig)
    x = mu + sig * rng.normal(size=(n, d))
    lq = f.log_prob(_dev(x)).cpu().numpy()
    _, lq_o = fl.forward(P, x, mu, sig)
    assert np.max(np.abs(lq - lq_o)) < 1e-12 * (1 + np.max(np.abs(lq_o)))
    z = rng.normal(size=(n, d))
    xs, lqs = f.sample(_dev(z))
    xo, lqo = fl.inverse(P, z, mu, sig)
    assert np.array_equal(xs.cpu().numpy(), xo)
    assert np.max(np.abs(lqs.cpu().numpy() - lqo)) < 1e-12 * (1 + np.max(np.abs(lqo)))
    f.close()


def test_whitened_identity_flow(lib):
    """Full lower-triangular whitening (x = Lw u + mu) with the identity flow: the exact
    Gaussian N(mu, Lw Lw^T) on both sides (1e-12)."""
    d, L, H, n = 14, 8, 256, 300
    rng = np.random.default_rng(31)
    A = rng.normal(size=(d, d))
    Lw = np.linalg.cholesky(A @ A.T + 0.01 * np.eye(d))
    mu = rng.normal(size=d) * 100.0
    P = fl.init_params(d, L, H, 5)
    f = lib.Flow(d, L, H, 512)
    f.set_params(lib.flow_pack(P), np.zeros(d), np.ones(d))
    f.set_whitening(mu, Lw)
    x = mu + rng.normal(size=(n, d)) @ Lw.T
    lq = f.log_prob(_dev(x)).cpu().numpy()
    _, lq_o = fl.forward(P, x, mu, Lw)
    assert np.max(np.abs(lq - lq_o)) < 1e-12 * (1 + np.max(np.abs(lq_o)))
    z = rng.normal(size=(n, d))
    xs, lqs = f.sample(_dev(z))
    xo, lqo = fl.inverse(P, z, mu, Lw)
    assert np.max(np.abs(xs.cpu().numpy() - xo)) < 1e-12 * np.max(np.abs(xo))
    assert np.max(np.abs(lqs.cpu().numpy() - lqo)) < 1e-12 * (1 + np.max(np.abs(lqo)))
    f.close()


@pytest.mark.parametrize("d,n", [(14, 300), (11, 1000), (2, 65)])
def test_flow_parity_bf16(lib, d, n):
    L, H = 8, 256
    rng = np.random.default_rng(d)
    P = _f32(_rand_params(d, L, H, d))
    mu, sig = rng.normal(size=d), rng.uniform(0.5, 3.0, size=d)
    f = lib.Flow(d, L, H, 1024)
    f.set_params(lib.flow_pack(P), mu, sig)
    x = mu + sig * rng.normal(size=(n, d))
    lq = f.log_prob(_dev(x)).cpu().numpy()
    _, lq_o = fl.forward(P, x, mu, sig)
    _, lq_b = bf16_ref.forward(P, x, mu, sig)
    assert np.max(np.abs(lq - lq_b)) < 1e-3
    assert np.all(np.abs(lq - lq_o) <= np.abs(lq_b - lq_o) + 1e-3)
    assert np.max(np.abs(lq - lq_o)) < 0.1
    zz = rng.normal(size=(n, d))
    xs, lqs = f.sample(_dev(zz))
    xs, lqs = xs.cpu().numpy(), lqs.cpu().numpy()
    xo, lqo = fl.inverse(P, zz, mu, sig)
    xb, lqb = bf16_ref.inverse(P, zz, mu, sig)
    # rounding-boundary flips of single BF16 operands leave rare larger outliers
    exb = np.abs((xs - xb) / sig)
    assert np.quantile(exb, 0.99) < 1e-6 and exb.max() < 5e-3
    assert np.max(np.abs(lqs - lqb)) < 1e-3
    assert np.all(np.abs(lqs - lqo) <= np.abs(lqb - lqo) + 1e-3)
    assert np.max(np.abs((xs - xo) / sig)) < 0.05
    # the library's own inverse and forward agree far below the BF16 level
    lq_back = f.log_prob(_dev(xs)).cpu().numpy()
    assert np.median(np.abs(lq_back - lqs)) < 1e-9 and np.max(np.abs(lq_back - lqs)) < 0.05
    f.close()


@pytest.mark.parametrize("d,n,H", [(14, 512, 256), (11, 37, 256), (5, 300, 64), (14, 1000, 96)])
def test_fused_coupling_bit_identical(lib, d, n, H):
    """Without gradients each coupling runs as one fused launch (products with h1, h2 in LDS);
    with gradients as separate launches that keep the activations.  Same operands, products,
    product order and rounding points: log q agrees bit for bit, over ragged row counts."""
    L = 8
    rng = np.random.default_rng(d + n)
    P = _f32(_rand_params(d, L, H, d + 7, scale=0.3))
    mu, sig = rng.normal(size=d), rng.uniform(0.5, 3.0, size=d)
    f = lib.Flow(d, L, H, 1024)
    f.set_params(lib.flow_pack(P), mu, sig)
    x = mu + sig * rng.normal(size=(n, d))
    fused = f.log_prob(_dev(x)).cpu().numpy()
    kept, _ = f.loss_grad(_dev(x))
    assert np.array_equal(fused, kept)
    f.close()


@pytest.mark.parametrize("d,n", [(14, 512), (5, 200)])
def test_gradient_parity(lib, d, n):
    L, H = 8, 256
    rng = np.random.default_rng(100 + d)
    P = _f32(_rand_params(d, L, H, 7 + d))
    mu, sig = rng.normal(size=d), rng.uniform(0.5, 2.0, size=d)
    f = lib.Flow(d, L, H, 1024)
    f.set_params(lib.flow_pack(P), mu, sig)
    x = mu + sig * rng.normal(size=(n, d)) * 1.3
    lq, g = f.loss_grad(_dev(x))
    loss_o, G = fl.nll_and_grad(P, x, mu, sig)
    Gb = bf16_ref.nll_grad(P, x, mu, sig)
    assert abs(-lq.mean() - loss_o) < 0.01
    Gg = lib.flow_unpack(g, d, L, H)

    def rel(a, b):
        return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-3)
    for l in range(L):
        for k in G[l]:
            assert rel(Gg[l][k], Gb[l][k]) < 0.01, (l, k)
            assert rel(Gg[l][k], G[l][k]) < max(0.1, 2 * rel(Gb[l][k], G[l][k])), (l, k)
    f.close()


def test_adam_step_parity(lib):
    d, L, H, n = 6, 4, 64, 256
    rng = np.random.default_rng(9)
    P = _f32(_rand_params(d, L, H, 4))
    mu, sig = np.zeros(d), np.ones(d)
    f = lib.Flow(d, L, H, n)
    w0 = lib.flow_pack(P)
    f.set_params(w0, mu, sig)
    x = rng.normal(size=(n, d))
    f.train(_dev(x), steps=1, batch=n, lr=1e-3)
    w1 = f.get_params()
    _, G = fl.nll_and_grad(P, x, mu, sig)
    opt = fl.Adam(P, lr=1e-3)
    opt.step(P, G)
    wo = lib.flow_pack(P)
    # first Adam step: each parameter moves by lr * g / (|g| + eps), i.e. by about +-lr
    dg, do = w1.astype(np.float64) - w0, wo.astype(np.float64) - w0
    close = np.abs(dg - do) < 2e-5
    assert close.mean() > 0.97
    f.close()


def test_trained_flow_matches_gaussian(lib):
    d, L, H = 4, 6, 128
    rng = np.random.default_rng(21)
    A = rng.normal(size=(d, d))
    C = A @ A.T + 0.5 * np.eye(d)
    m = np.array([1.0, -2.0, 3.0, 0.0])
    x = rng.multivariate_normal(m, C, size=20000)
    f = lib.Flow(d, L, H, 1024)
    f.set_params(lib.flow_pack(fl.init_params(d, L, H, 2)), x.mean(0), x.std(0))
    f.train(_dev(x), steps=1500, batch=1024, lr=2e-3)
    xs, _ = f.sample(_dev(rng.normal(size=(1024, d))))
    xs = xs.cpu().numpy()
    assert np.allclose(xs.mean(0), m, atol=0.2 * np.sqrt(np.diag(C)).max())
    assert np.allclose(np.cov(xs.T), C, atol=0.2 * np.abs(C).max())
    exact = -0.5 * np.einsum("ni,ij,nj->n", x - m, np.linalg.inv(C), x - m) - 0.5 * np.log(np.linalg.det(2 * np.pi * C))
    lq = f.log_prob(_dev(x[:1024])).cpu().numpy()
    assert abs(lq.mean() - exact[:1024].mean()) < 0.1
    # parity of the trained flow with the oracle evaluated on the same FP32 weights
    P = lib.flow_unpack(f.get_params(), d, L, H)
    _, lq_o = fl.forward(P, x[:1024], x.mean(0), x.std(0))
    _, lq_b = bf16_ref.forward(P, x[:1024], x.mean(0), x.std(0))
    assert np.max(np.abs(lq - lq_b)) < 1e-3
    # against FP64: each row no further than the BF16 model of the library is itself (+1e-3)
    assert np.max(np.abs(lq - lq_o) - np.abs(lq_b - lq_o)) < 1e-3
    f.close()


@pytest.mark.parametrize("T,full,mb", [(1, False, 1), (2, False, 1), (2, True, 1), (2, False, 2), (2, True, 2)])
def test_sampler_flow_move_parity(lib, T, full, mb):
    """P28: GPU chain with an (exact, identity) flow move against the oracle chain, step by step.
    mb = 2: the flow holds twice the walkers, so the proposals and the log q of the current
    positions go through its passes together (one launch per layer for both)."""
    d, W, seed = 5, 16, 777
    rng = np.random.default_rng(T)
    A = rng.normal(size=(d, d))
    icov = np.linalg.inv(A @ A.T + d * np.eye(d))
    means = rng.normal(size=(1, d))
    lo, hi = -30 * np.ones(d), 30 * np.ones(d)
    P = fl.init_params(d, 4, 32, 1)
    mu, sig = means[0] + 0.5, np.linspace(1.0, 3.0, d)
    start = means[0] + rng.normal(size=(T, W, d))
    fg = lib.Flow(d, 4, 32, mb * W)
    fg.set_params(lib.flow_pack(P), mu, sig)
    if full:                 # whitening by the target's own Cholesky factor (scaled up by 1.2)
        sig = 1.2 * np.linalg.cholesky(np.linalg.inv(icov))
        fg.set_whitening(mu, sig)
    g = lib.Sampler(W, T, d, lo, hi, seed, target="gauss", param_kind="raw", t_max=5.0, means=means, icov=icov)
    g.set_flow(fg)
    g.set_state(start)
    o = PTSampler(gaussian_logl(means, icov), lo, hi, W, T, d, seed, t_max=5.0)
    o.set_flow(P, mu, sig)
    o.set_state(start)
    for s in range(25):
        g.step(1)
        o.step()
        pos, logl, _, step, cnt = g.state()
        assert np.max(np.abs(pos - o.X)) < 1e-12 * (1 + np.max(np.abs(o.X))), s
        assert cnt[0] == o.acc and cnt[2] == o.sacc
        assert g.flow_counts() == (o.facc, o.fprop), s
    assert 0 < o.facc < o.fprop
    g.close()
    fg.close()


@pytest.mark.gpu
@pytest.mark.parametrize("p_flow", [0.0, 0.35])
def test_sampler_flow_mix_parity(lib, p_flow):
    """P36: the flow move mixed with the stretch move at rate p_flow (a Philox draw per step on
    the device) against the oracle chain, step by step; p_flow = 0 is the plain sampler."""
    d, W, T, seed = 4, 16, 2, 4242
    rng = np.random.default_rng(9)
    A = rng.normal(size=(d, d))
    icov = np.linalg.inv(A @ A.T + d * np.eye(d))
    means = rng.normal(size=(1, d))
    lo, hi = -30 * np.ones(d), 30 * np.ones(d)
    P = fl.init_params(d, 4, 32, 2)
    mu, sig = means[0] - 0.4, np.linspace(1.5, 2.5, d)
    start = means[0] + rng.normal(size=(T, W, d))
    fg = lib.Flow(d, 4, 32, W)
    fg.set_params(lib.flow_pack(P), mu, sig)
    g = lib.Sampler(W, T, d, lo, hi, seed, target="gauss", param_kind="raw", t_max=5.0, means=means, icov=icov)
    g.set_flow(fg)
    g.set_flow_mix(p_flow)
    g.set_state(start)
    o = PTSampler(gaussian_logl(means, icov), lo, hi, W, T, d, seed, t_max=5.0)
    o.set_flow(P, mu, sig)
    o.set_flow_mix(p_flow)
    o.set_state(start)
    for s in range(40):
        g.step(1)
        o.step()
        pos, logl, _, step, cnt = g.state()
        assert np.max(np.abs(pos - o.X)) < 1e-12 * (1 + np.max(np.abs(o.X))), s
        assert cnt[0] == o.acc and cnt[2] == o.sacc
        assert g.flow_counts() == (o.facc, o.fprop), s
    if p_flow > 0:
        assert 0 < o.flow_steps < 40 and 0 < o.facc
    else:
        assert o.fprop == 0
    with pytest.raises(lib.LisaTDError):
        g.set_flow_mix(1.5)
    g.close()
    fg.close()


@pytest.mark.gpu
@pytest.mark.parametrize("T", [1, 2])
def test_sampler_flow_exclusive_parity(lib, T):
    """P37: on the flow move's steps the cold rung skips its stretch moves; the GPU chain, the
    stretch, swap and flow counts match the oracle's step by step."""
    d, W, seed = 4, 16, 4243
    rng = np.random.default_rng(11)
    A = rng.normal(size=(d, d))
    icov = np.linalg.inv(A @ A.T + d * np.eye(d))
    means = rng.normal(size=(1, d))
    lo, hi = -30 * np.ones(d), 30 * np.ones(d)
    P = fl.init_params(d, 4, 32, 3)
    mu, sig = means[0] + 0.3, np.linspace(1.2, 2.2, d)
    start = means[0] + rng.normal(size=(T, W, d))
    fg = lib.Flow(d, 4, 32, W)
    fg.set_params(lib.flow_pack(P), mu, sig)
    g = lib.Sampler(W, T, d, lo, hi, seed, target="gauss", param_kind="raw", t_max=5.0, means=means, icov=icov)
    g.set_flow(fg)
    g.set_flow_mix(0.5)
    g.set_flow_exclusive(True)
    g.set_state(start)
    o = PTSampler(gaussian_logl(means, icov), lo, hi, W, T, d, seed, t_max=5.0)
    o.set_flow(P, mu, sig)
    o.set_flow_mix(0.5)
    o.set_flow_exclusive(True)
    o.set_state(start)
    for s in range(40):
        g.step(1)
        o.step()
        pos, logl, _, step, cnt = g.state()
        assert np.max(np.abs(pos - o.X)) < 1e-12 * (1 + np.max(np.abs(o.X))), s
        assert (cnt[0], cnt[1], cnt[2]) == (o.acc, o.prop, o.sacc), s
        assert g.flow_counts() == (o.facc, o.fprop), s
    assert 0 < o.flow_steps < 40 and o.prop == 40 * T * W - o.flow_steps * W
    with pytest.raises(lib.LisaTDError):
        lib._check(lib._lib.lt_sampler_set_flow_exclusive(g.h, 2))
    g.close()
    fg.close()


@pytest.mark.gpu
@pytest.mark.parametrize("T,excl", [(1, False), (2, True)])
def test_sampler_flow_mixture_parity(lib, T, excl):
    """P38: a mixture of two flows as the proposal (component per walker from Philox, mixture
    density at both ends) against the oracle chain, step by step, on a two-mode Gaussian whose
    walkers start in one mode; the chain reaches the other through the second flow."""
    d, W, seed = 3, 16, 4244
    means = np.array([[-6.0, 0.5, 0.0], [6.0, -0.5, 1.0]])
    icov = np.eye(d)
    lo, hi = -40 * np.ones(d), 40 * np.ones(d)
    rng = np.random.default_rng(12)
    start = means[0] + rng.normal(size=(T, W, d))
    P1, P2 = fl.init_params(d, 2, 32, 4), fl.init_params(d, 2, 32, 5)
    mu1, s1 = means[0] + 0.2, np.array([1.3, 1.2, 1.1])
    mu2, s2 = means[1] - 0.1, np.array([1.2, 1.4, 1.0])
    f1, f2 = lib.Flow(d, 2, 32, W), lib.Flow(d, 2, 32, W)
    f1.set_params(lib.flow_pack(P1), mu1, s1)
    f2.set_params(lib.flow_pack(P2), mu2, s2)
    g = lib.Sampler(W, T, d, lo, hi, seed, target="gauss", param_kind="raw", t_max=5.0, means=means, icov=icov)
    g.set_flow(f1)
    g.set_flow_mixture(f2, 0.4)
    g.set_flow_exclusive(excl)
    g.set_state(start)
    o = PTSampler(gaussian_logl(means, icov), lo, hi, W, T, d, seed, t_max=5.0)
    o.set_flow(P1, mu1, s1)
    o.set_flow_mixture(P2, mu2, s2, 0.4)
    o.set_flow_exclusive(excl)
    o.set_state(start)
    for st in range(40):
        g.step(1)
        o.step()
        pos, logl, _, step, cnt = g.state()
        assert np.max(np.abs(pos - o.X)) < 1e-12 * (1 + np.max(np.abs(o.X))), st
        assert (cnt[0], cnt[1], cnt[2]) == (o.acc, o.prop, o.sacc), st
        assert g.flow_counts() == (o.facc, o.fprop), st
    assert np.mean(o.X[0, :, 0] > 0) > 0.2    # the second mode is reached
    with pytest.raises(lib.LisaTDError):
        g.set_flow_mixture(f2, 1.0)
    with pytest.raises(lib.LisaTDError):
        g.set_flow_walk(0.1)
    g.close()
    f1.close()
    f2.close()


@pytest.mark.gpu
@pytest.mark.parametrize("T", [1, 3])
def test_sampler_flow_fold_parity(lib, T):
    """P29: flow move with the symmetry fold (copies drawn from Philox, -ln n corrections,
    proposals outside the window rejected) against the oracle chain, step by step, on a
    two-mode Gaussian whose modes sit one period apart in the folded coordinate; the copy
    count varies over the range."""
    d, W, seed, i, Pd, c0 = 4, 16, 4242, 2, 2.0, -1.0
    rng = np.random.default_rng(10 + T)
    A = rng.normal(size=(d, d))
    icov = np.linalg.inv(0.05 * (A @ A.T) + 0.2 * np.eye(d))
    m = rng.normal(size=d)
    m[i] = 0.1
    means = np.stack([m, m + Pd * np.eye(d)[i]])
    lo, hi = -30 * np.ones(d), 30 * np.ones(d)
    lo[i], hi[i] = -1.7, 2.6
    P = fl.init_params(d, 4, 32, 1)
    mu, sig = m + 0.1, np.full(d, 0.7)
    start = np.clip(means[0] + 0.3 * rng.normal(size=(T, W, d)), lo + 1e-3, hi - 1e-3)
    fg = lib.Flow(d, 4, 32, W)
    fg.set_params(lib.flow_pack(P), mu, sig)
    g = lib.Sampler(W, T, d, lo, hi, seed, target="gauss", param_kind="raw", t_max=5.0, means=means, icov=icov)
    g.set_flow(fg)
    g.set_flow_fold(i, Pd, c0)
    g.set_state(start)
    o = PTSampler(gaussian_logl(means, icov), lo, hi, W, T, d, seed, t_max=5.0)
    o.set_flow(P, mu, sig)
    o.set_flow_fold(i, Pd, c0)
    o.set_state(start)
    for s in range(25):
        g.step(1)
        o.step()
        pos, logl, _, step, cnt = g.state()
        assert np.max(np.abs(pos - o.X)) < 1e-12 * (1 + np.max(np.abs(o.X))), s
        assert cnt[0] == o.acc and cnt[2] == o.sacc
        assert g.flow_counts() == (o.facc, o.fprop), s
    assert 0 < o.facc < o.fprop
    assert np.any(o.X[0, :, i] > c0 + Pd) or np.any(o.X[0, :, i] < c0)   # some walker sits on another copy
    g.close()
    fg.close()


@pytest.mark.gpu
@pytest.mark.parametrize("fold", [False, True])
def test_sampler_flow_walk_parity(lib, fold):
    """P30: the latent random-walk flow move (walk normals from Philox, log q - log N at both
    ends), with and without the symmetry fold, against the oracle chain step by step."""
    d, W, T, seed, i, Pd, c0 = 4, 16, 2, 5151, 2, 2.0, -1.0
    rng = np.random.default_rng(40 + fold)
    A = rng.normal(size=(d, d))
    icov = np.linalg.inv(0.05 * (A @ A.T) + 0.2 * np.eye(d))
    m = rng.normal(size=d)
    m[i] = 0.1
    means = np.stack([m, m + Pd * np.eye(d)[i]])
    lo, hi = -30 * np.ones(d), 30 * np.ones(d)
    lo[i], hi[i] = -1.7, 2.6
    P = fl.init_params(d, 4, 32, 3)
    mu, sig = m + 0.1, np.full(d, 0.7)
    start = np.clip(means[0] + 0.3 * rng.normal(size=(T, W, d)), lo + 1e-3, hi - 1e-3)
    fg = lib.Flow(d, 4, 32, W)
    fg.set_params(lib.flow_pack(P), mu, sig)
    g = lib.Sampler(W, T, d, lo, hi, seed, target="gauss", param_kind="raw", t_max=5.0, means=means, icov=icov)
    o = PTSampler(gaussian_logl(means, icov), lo, hi, W, T, d, seed, t_max=5.0)
    g.set_flow(fg)
    o.set_flow(P, mu, sig)
    if fold:
        g.set_flow_fold(i, Pd, c0)
        o.set_flow_fold(i, Pd, c0)
    g.set_flow_walk(0.6)
    o.set_flow_walk(0.6)
    g.set_state(start)
    o.set_state(start)
    for s in range(25):
        g.step(1)
        o.step()
        pos, logl, _, step, cnt = g.state()
        assert np.max(np.abs(pos - o.X)) < 1e-12 * (1 + np.max(np.abs(o.X))), s
        assert cnt[0] == o.acc and cnt[2] == o.sacc
        assert g.flow_counts() == (o.facc, o.fprop), s
    assert 0 < o.facc < o.fprop
    g.close()
    fg.close()


def test_learned_proposal_raises_ess(lib):
    """A flow trained on burn-in samples lowers the cold chain's integrated autocorrelation time."""
    d, W = 4, 64
    rng = np.random.default_rng(5)
    A = rng.normal(size=(d, d))
    C = A @ A.T + 0.05 * np.eye(d)          # strongly correlated
    means = np.zeros((1, d))
    icov = np.linalg.inv(C)
    lo, hi = -60 * np.ones(d), 60 * np.ones(d)
    start = rng.multivariate_normal(means[0], C, size=(1, W))

    def run(flow, steps):
        s = lib.Sampler(W, 1, d, lo, hi, 99, target="gauss", param_kind="raw", means=means, icov=icov)
        if flow is not None:
            s.set_flow(flow)
        s.set_state(start)
        chain = []
        for _ in range(steps):
            s.step(1)
            chain.append(s.state()[0][0])
        s.close()
        return np.array(chain)

    plain = run(None, 1200)
    burn = plain[200:].reshape(-1, d)
    f = lib.Flow(d, 6, 128, 1024)
    f.set_params(lib.flow_pack(fl.init_params(d, 6, 128, 0)), burn.mean(0), burn.std(0))
    xs = burn[rng.permutation(len(burn))]
    f.train(_dev(xs), steps=1000, batch=1024, lr=2e-3)
    learned = run(f, 1200)
    tau_plain = integrated_time(plain[200:]).max()
    tau_flow = integrated_time(learned[200:]).max()
    assert tau_flow < 0.5 * tau_plain, (tau_flow, tau_plain)
    flat = learned[200:].reshape(-1, d)
    assert np.allclose(np.cov(flat.T), C, atol=0.15 * np.abs(C).max())
    f.close()
