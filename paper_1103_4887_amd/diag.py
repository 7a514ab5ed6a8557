"""Chain diagnostics: effective sample size and Monte Carlo standard error.

Measurement tooling, not part of the sampler: ESS by Geyer's initial
monotone sequence estimator (Geyer 1992, "Practical Markov chain Monte
Carlo"), MCSE = sd / sqrt(ESS), batch-means MCSE.
"""

from __future__ import annotations

import numpy as np


def autocorr(x: np.ndarray) -> np.ndarray:
    """Normalised autocorrelation rho_k, k = 0..n-1 (FFT, biased estimator)."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    d = x - x.mean()
    m = 1 << (2 * n - 1).bit_length()
    f = np.fft.rfft(d, m)
    ac = np.fft.irfft(f * np.conj(f), m)[:n]
    if ac[0] <= 0:
        return np.zeros(n)
    return ac / ac[0]


def ess(x: np.ndarray) -> float:
    """Effective sample size of one scalar chain (initial monotone sequence)."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    if n < 4:
        return float(n)
    if np.all(x == x[0]):
        return 0.0
    rho = autocorr(x)
    npairs = n // 2
    gam = rho[0:2 * npairs:2] + rho[1:2 * npairs:2]
    s = 0.0
    prev = np.inf
    for g in gam:
        if g <= 0:
            break
        g = min(g, prev)
        s += g
        prev = g
    tau = -1.0 + 2.0 * s
    tau = max(tau, 1.0 / np.log10(max(n, 10)))
    return float(n / tau)


def ess_columns(trace: np.ndarray) -> np.ndarray:
    """ESS of every column of a (n, k) trace."""
    return np.array([ess(trace[:, j]) for j in range(trace.shape[1])])


def mcse(x: np.ndarray) -> float:
    e = ess(x)
    return float(np.std(x, ddof=1) / np.sqrt(max(e, 1.0)))


def batch_mcse(trace: np.ndarray, nb: int = 32) -> np.ndarray:
    """MCSE of the mean from nb batch means, for each column of a trace."""
    n = trace.shape[0] // nb * nb
    b = trace[:n].reshape(nb, -1, *trace.shape[1:]).mean(axis=1)
    return b.std(axis=0, ddof=1) / np.sqrt(nb)
