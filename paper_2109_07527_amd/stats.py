"""Time-series statistics for Monte Carlo output (host-side, numpy).

* ``tau_int``      - integrated autocorrelation time with Sokal's automatic
                     windowing (window M = smallest M with M >= c * tau(M)).
* ``blocking_se``  - standard error of the mean by Flyvbjerg-Petersen blocking
                     (plateau of the blocked estimate, taken as its maximum over
                     levels that keep at least 32 blocks).
* ``mean_se``      - mean and standard error using tau_int.
"""
from __future__ import annotations

import math

import numpy as np


def autocorrelation(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    x = x - x.mean()
    f = np.fft.rfft(x, n=2 * n)
    acf = np.fft.irfft(f * np.conj(f))[:n]
    if acf[0] <= 0:
        return np.zeros(n)
    return acf / acf[0]


def tau_int(x: np.ndarray, c: float = 5.0) -> float:
    """Integrated autocorrelation time (in samples), tau = 1/2 + sum_{t>=1} rho(t)."""
    rho = autocorrelation(x)
    n = rho.size
    if n < 4 or not np.isfinite(rho).all() or rho[0] == 0:
        return 0.5
    tau = 0.5
    for m in range(1, n):
        tau += rho[m]
        if m >= c * tau:
            break
    return max(float(tau), 0.5)


def mean_se(x: np.ndarray, c: float = 5.0):
    x = np.asarray(x, dtype=np.float64)
    t = tau_int(x, c)
    var = x.var(ddof=1) if x.size > 1 else 0.0
    return float(x.mean()), math.sqrt(2.0 * t * var / max(x.size, 1)), t


def blocking_se(x: np.ndarray) -> float:
    x = np.asarray(x, dtype=np.float64)
    best = 0.0
    while x.size >= 32:
        se = math.sqrt(x.var(ddof=1) / x.size)
        best = max(best, se)
        m = x.size // 2
        x = 0.5 * (x[: 2 * m : 2] + x[1 : 2 * m : 2])
    return best
