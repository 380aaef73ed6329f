"""Integrated autocorrelation time and effective sample size of a Monte Carlo series.

tau_int(W) = 1/2 + sum_{t=1..W} rho(t), rho(t) the normalised autocovariance;
the window W is the smallest with W >= c * tau_int(W), c = 5 (Sokal's automatic
windowing, in "Monte Carlo methods in statistical mechanics", 1997).  The error
estimate is tau * sqrt(2 (2W + 1) / N) (Madras-Sokal).  ESS = N / (2 tau_int).
"""
from __future__ import annotations

import numpy as np


def autocov(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, float) - np.mean(x)
    n = len(x)
    return np.array([np.dot(x[:n - t], x[t:]) / n for t in range(n)])


def tau_int(x, c: float = 5.0):
    """(tau, tau_err, window) of a 1-D series."""
    x = np.asarray(x, float)
    n = len(x)
    g = autocov(x)
    if g[0] <= 0:
        return 0.5, 0.0, 0
    rho = g / g[0]
    tau = 0.5
    w = 0
    for t in range(1, n):
        tau += rho[t]
        w = t
        if t >= c * tau:
            break
    tau = max(tau, 0.5)
    err = tau * np.sqrt(2.0 * (2 * w + 1) / n)
    return tau, err, w


def tau_int_chains(x, c: float = 5.0):
    """(tau, tau_err, window) of several independent series x[t, s] of one chain ensemble: each
    series centred on its own mean, the autocovariances averaged over series, then the same
    windowed sum as ``tau_int``; the error uses all n_t * n_series samples."""
    x = np.asarray(x, float)
    n, m = x.shape
    g = np.mean([autocov(x[:, s]) for s in range(m)], axis=0)
    if g[0] <= 0:
        return 0.5, 0.0, 0
    rho = g / g[0]
    tau = 0.5
    w = 0
    for t in range(1, n):
        tau += rho[t]
        w = t
        if t >= c * tau:
            break
    tau = max(tau, 0.5)
    err = tau * np.sqrt(2.0 * (2 * w + 1) / (n * m))
    return tau, err, w


def ess(x, c: float = 5.0) -> float:
    tau, _, _ = tau_int(x, c)
    return len(x) / (2.0 * tau)
