"""Closed-form posterior of the D=1 linear-Gaussian window (a pin).

For dx/dt = -lam x + I(t) the trapezoid model error of Section 2.1 is affine
in the path: eps_n = a x_n - b x_{n-1} - k_n with a = 1 + lam dt/2,
b = 1 - lam dt/2, k_n = dt/2 (I_n + I_{n-1}).  With a flat prior on x_0 the
path posterior exp(-A) is Gaussian (Section 1: the Kalman solution is exact
in this case) with tridiagonal precision

  Q_00 = beta Rd b^2,  Q_nn = beta Rd (a^2 + b^2) + Ro (1 <= n <= M-1),
  Q_MM = beta Rd a^2 + Ro,  Q_{n,n-1} = -beta Rd a b,

and mean Q^{-1} g, g_n = beta Rd a k_n [n>=1] - beta Rd b k_{n+1} [n<=M-1]
+ Ro y_n [n>=1].  `rts_smoother` derives the same moments a second way, as
a forward Kalman filter plus Rauch-Tung-Striebel backward pass.
"""

from __future__ import annotations

import numpy as np
from scipy.linalg import solveh_banded


def _coeffs(spec, I, lam):
    dt = spec.dt
    a = 1.0 + 0.5 * lam * dt
    b = 1.0 - 0.5 * lam * dt
    k = np.zeros(len(I))
    k[1:] = 0.5 * dt * (I[1:] + I[:-1])
    return a, b, k


def lin1_posterior(spec, y, I, lam, prior_var=None):
    """(mean, var) of every x_n under exp(-A), from the tridiagonal precision.

    prior_var=None is the flat prior on x_0 of the sampler; a number adds a
    N(0, prior_var) prior on x_0 (to compare with the smoother exactly)."""
    M = len(y) - 1
    a, b, k = _coeffs(spec, np.asarray(I, dtype=np.float64), lam)
    R = spec.beta * spec.Rd[0]
    Ro = spec.Ro
    diag = np.empty(M + 1)
    diag[0] = R * b * b
    diag[1:M] = R * (a * a + b * b) + Ro
    diag[M] = R * a * a + Ro
    if prior_var is not None:
        diag[0] += 1.0 / prior_var
    off = np.full(M, -R * a * b)
    g = np.zeros(M + 1)
    g[1:] += R * a * k[1:] + Ro * np.asarray(y[1:])
    g[:-1] += -R * b * k[1:]
    ab = np.zeros((2, M + 1))
    ab[0, 1:] = off
    ab[1] = diag
    mean = solveh_banded(ab, g)
    Q = np.diag(diag) + np.diag(off, 1) + np.diag(off, -1)
    var = np.diag(np.linalg.inv(Q)).copy()
    return mean, var


def rts_smoother(spec, y, I, lam, prior_var=1e6):
    """Kalman filter + RTS smoother of x_n = (b x_{n-1} + k_n + e_n) / a."""
    M = len(y) - 1
    a, b, k = _coeffs(spec, np.asarray(I, dtype=np.float64), lam)
    q = 1.0 / (spec.beta * spec.Rd[0] * a * a)   # var of e_n / a
    r = 1.0 / spec.Ro
    F = b / a
    mf = np.zeros(M + 1)
    Pf = np.zeros(M + 1)
    mp_ = np.zeros(M + 1)
    Pp = np.zeros(M + 1)
    mf[0], Pf[0] = 0.0, prior_var
    for n in range(1, M + 1):
        mp_[n] = F * mf[n - 1] + k[n] / a
        Pp[n] = F * F * Pf[n - 1] + q
        # update written without 1 - K, which cancels for a diffuse prior
        mf[n] = (r * mp_[n] + Pp[n] * y[n]) / (Pp[n] + r)
        Pf[n] = Pp[n] * r / (Pp[n] + r)
    ms = mf.copy()
    Ps = Pf.copy()
    for n in range(M - 1, -1, -1):
        C = Pf[n] * F / Pp[n + 1]
        ms[n] = mf[n] + C * (ms[n + 1] - mp_[n + 1])
        Ps[n] = Pf[n] + C * C * (Ps[n + 1] - Pp[n + 1])
    return ms, Ps
