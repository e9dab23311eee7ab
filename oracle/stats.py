"""Oracle for the integrated autocorrelation time (test infrastructure only).

Plain numpy, fp64, straight from the definitions: the grand mean over all
chains and samples is removed (so chains stuck at different levels show up
as correlation that does not decay, as it should for an effective sample
size of the target law), the autocovariance at lag k is summed over chains
and normalised by (n - k) and the number of chains, rho(k) = Gamma(k) /
Gamma(0), tau_int(W) = 1 + 2 sum_{k<=W} rho(k), automatic window
W = min{W : W >= c tau_int(W)} (Sokal, "Monte Carlo methods in statistical
mechanics", 1996), else the largest lag; ESS = chains * samples / tau_int.
"""
import numpy as np


def autocorr(x):
    """x: [n_samples, n_chains] float64 -> rho(k), k = 0..n-1."""
    x = np.asarray(x, np.float64)
    n, nc = x.shape
    y = x - x.mean()
    gam = np.empty(n)
    for k in range(n):
        gam[k] = (y[: n - k] * y[k:]).sum() / (n - k) / nc
    return gam / gam[0] if gam[0] > 0 else np.where(np.arange(n) == 0, 1.0, 0.0)


def tau_int(x, max_lag=2000, c=6.0):
    x = np.asarray(x, np.float64)
    n, nc = x.shape
    rho = autocorr(x)[: min(max_lag, n - 1) + 1]
    tau, W = 1.0, len(rho) - 1
    for k in range(1, len(rho)):
        tau += 2.0 * rho[k]
        if k >= c * tau:
            W = k
            break
    return tau, nc * n / tau, W, rho
