"""Chain diagnostics on the host: integrated autocorrelation time and
effective sample size of ensemble chains (used to report ESS/s)."""
import numpy as np


def autocorr_time(chain, window=5.0):
    """chain [steps][walkers][dim] -> integrated autocorrelation time per
    coordinate.  The normalised autocovariance of each walker (FFT, zero
    padded to 2 x steps) is averaged over walkers, tau(M) = 1 + 2 sum_{1..M}
    rho, and M is the first lag with M >= window * tau(M) (Sokal)."""
    x = np.asarray(chain, dtype=np.float64)
    n = x.shape[0]
    x = x - x.mean(axis=0, keepdims=True)
    f = np.fft.rfft(x, n=2 * n, axis=0)
    acov = np.fft.irfft(f * np.conj(f), axis=0)[:n]
    var = acov[0]
    ok = var > 0
    rho = np.where(ok, acov / np.where(ok, var, 1.0), 0.0)
    counted = np.maximum(ok.sum(axis=0), 1)
    rho = rho.sum(axis=1) / counted                     # [lags][dim]
    tau = 2.0 * np.cumsum(rho, axis=0) - 1.0
    lags = np.arange(n)[:, None]
    stop = lags >= window * tau
    first = np.where(stop.any(axis=0), stop.argmax(axis=0), n - 1)
    return tau[first, np.arange(tau.shape[1])]


def ess(chain, window=5.0):
    """Effective samples of the worst coordinate: steps x walkers / max tau."""
    x = np.asarray(chain)
    return x.shape[0] * x.shape[1] / float(np.max(autocorr_time(x, window)))


def _batches(chain, n_batches):
    x = np.asarray(chain, dtype=np.float64)
    L = x.shape[0] // n_batches
    if L < 1:
        raise ValueError("fewer steps than batches")
    return x[:L * n_batches].reshape(n_batches, L, *x.shape[1:])


def batch_ess(chain, n_batches=20):
    """Effective samples per coordinate from batch means of the whole ensemble: the chain
    [steps][walkers][dim] is cut into n_batches runs of consecutive steps, each run's mean over
    all its steps and walkers is one batch mean, and ESS = n_batches var(x) / var(batch means).
    Unlike autocorr_time, which removes each walker's own mean, this sees correlation between
    walkers (a coupled ensemble, or one that drifts as a whole) as well as along the chain.
    Capped at the number of samples."""
    b = _batches(chain, n_batches)
    bm = b.mean(axis=(1, 2))
    var_x = b.reshape(-1, b.shape[-1]).var(axis=0)
    var_bm = bm.var(axis=0, ddof=1)
    n = b.shape[0] * b.shape[1] * b.shape[2]
    return np.minimum(n_batches * var_x / np.maximum(var_bm, 1e-300), n)


def batch_quantile_se(chain, qs=(0.05, 0.5, 0.95), n_batches=20):
    """Quantiles of each coordinate's marginal [len(qs)][dim] and their Monte-Carlo standard
    errors from the spread of the same quantiles over n_batches runs of consecutive steps."""
    x = np.asarray(chain, dtype=np.float64)
    b = _batches(x, n_batches)
    q = np.quantile(x.reshape(-1, x.shape[-1]), qs, axis=0)
    qb = np.stack([np.quantile(bb.reshape(-1, bb.shape[-1]), qs, axis=0) for bb in b])
    return q, qb.std(axis=0, ddof=1) / np.sqrt(n_batches)
