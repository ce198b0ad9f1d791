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
