"""Vector fields F(x; p), Jacobians and parameter derivatives (oracle, FP64).

HH (Section 5.1): x = (V, m, h, n),
  dV/dt = p1 I + p2 m^3 h (p3 - V) + p4 n^4 (p5 - V) + p6 (p7 - V)
  da/dt = (a_inf(V) - a) / tau_a(V),  a in {m, h, n}
  a_inf = 1/2 + 1/2 tanh(s),  tau_a = tau0 + tau1 (1 - tanh(s)^2),
  s = (V - V_a) / dV_a, with (V_a, dV_a, tau0, tau1) from Table 1.

LIN1 (the D=1 linear-Gaussian test window): dx/dt = -p1 x + I.

All functions take arrays over sites: X (N, D), I (N,), p (Np,).
"""

from __future__ import annotations

import numpy as np


class HH:
    D = 4
    Np = 7

    def __init__(self, gates):
        # gates: ((V_a, dV_a, tau0, tau1) for m, h, n)
        self.g = np.asarray(gates, dtype=np.float64)

    def _gate(self, V, j):
        Va, dVa, t0, t1 = self.g[j]
        t = np.tanh((V - Va) / dVa)
        return t, 0.5 + 0.5 * t, t0 + t1 * (1.0 - t * t)

    def F(self, X, I, p):
        V, m, h, n = X[:, 0], X[:, 1], X[:, 2], X[:, 3]
        out = np.empty_like(X, dtype=np.float64)
        out[:, 0] = (p[0] * I + p[1] * m ** 3 * h * (p[2] - V)
                     + p[3] * n ** 4 * (p[4] - V) + p[5] * (p[6] - V))
        for j, a in enumerate((m, h, n)):
            _, ainf, tau = self._gate(V, j)
            out[:, 1 + j] = (ainf - a) / tau
        return out

    def J(self, X, p):
        """dF_a/dx_b, shape (N, 4, 4); row = component of F."""
        V, m, h, n = X[:, 0], X[:, 1], X[:, 2], X[:, 3]
        N = X.shape[0]
        Jm = np.zeros((N, 4, 4))
        Jm[:, 0, 0] = -(p[1] * m ** 3 * h + p[3] * n ** 4 + p[5])
        Jm[:, 0, 1] = 3.0 * p[1] * m ** 2 * h * (p[2] - V)
        Jm[:, 0, 2] = p[1] * m ** 3 * (p[2] - V)
        Jm[:, 0, 3] = 4.0 * p[3] * n ** 3 * (p[4] - V)
        for j, a in enumerate((m, h, n)):
            Va, dVa, t0, t1 = self.g[j]
            t, ainf, tau = self._gate(V, j)
            dt_dV = (1.0 - t * t) / dVa          # d tanh(s)/dV
            dainf = 0.5 * dt_dV
            dtau = -2.0 * t1 * t * dt_dV
            Jm[:, 1 + j, 0] = dainf / tau - (ainf - a) * dtau / (tau * tau)
            Jm[:, 1 + j, 1 + j] = -1.0 / tau
        return Jm

    def dF_dp(self, X, I, p):
        """dF/dp, shape (N, 4, 7); only the V row is non-zero."""
        V, m, h, n = X[:, 0], X[:, 1], X[:, 2], X[:, 3]
        N = X.shape[0]
        d = np.zeros((N, 4, 7))
        d[:, 0, 0] = I
        d[:, 0, 1] = m ** 3 * h * (p[2] - V)
        d[:, 0, 2] = p[1] * m ** 3 * h
        d[:, 0, 3] = n ** 4 * (p[4] - V)
        d[:, 0, 4] = p[3] * n ** 4
        d[:, 0, 5] = p[6] - V
        d[:, 0, 6] = p[5]
        return d


class Lin1:
    D = 1
    Np = 1

    def F(self, X, I, p):
        return (-p[0] * X[:, 0] + I)[:, None]

    def J(self, X, p):
        return np.full((X.shape[0], 1, 1), -p[0])

    def dF_dp(self, X, I, p):
        return (-X[:, 0])[:, None, None]


def model_for(spec):
    """Oracle model object for a workloads.ModelSpec."""
    if spec.kind == "hh":
        return HH(spec.gates)
    if spec.kind == "lin1":
        return Lin1()
    raise ValueError(f"unknown model kind {spec.kind!r}")
