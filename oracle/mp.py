"""High-precision (mpmath, 50 digits) action for tiny windows: a pin.

Evaluates the same definitions as `action.action` (Section 2.1; HH field of
Section 5.1) term by term in 50-digit arithmetic with mpmath's own tanh, so a
dropped term, a wrong sign or a wrong index in the FP64 code shows up as a
disagreement far above FP64 rounding.
"""

from __future__ import annotations

import mpmath as mp


def _F_hh(x, I, p, gates):
    V, m, h, n = x
    out = [p[0] * I + p[1] * m ** 3 * h * (p[2] - V) + p[3] * n ** 4 * (p[4] - V) + p[5] * (p[6] - V)]
    for a, (Va, dVa, t0, t1) in zip((m, h, n), gates):
        t = mp.tanh((V - mp.mpf(Va)) / mp.mpf(dVa))
        out.append((mp.mpf(0.5) + t / 2 - a) / (mp.mpf(t0) + mp.mpf(t1) * (1 - t * t)))
    return out


def _F_lin1(x, I, p):
    return [-p[0] * x[0] + I]


def action_mp(spec, X, y, I, p, dps: int = 50):
    with mp.workdps(dps):
        mpf = mp.mpf
        Xm = [[mpf(float(v)) for v in row] for row in X]
        Im = [mpf(float(v)) for v in I]
        pm = [mpf(float(v)) for v in p]
        if spec.kind == "hh":
            F = [_F_hh(Xm[n], Im[n], pm, spec.gates) for n in range(len(Xm))]
        else:
            F = [_F_lin1(Xm[n], Im[n], pm) for n in range(len(Xm))]
        h = mpf(float(spec.dt)) / 2
        A_o = mpf(0)
        A_d = mpf(0)
        for n in range(1, len(Xm)):
            d = mpf(float(y[n])) - Xm[n][0]
            A_o += mpf(float(spec.Ro)) * d * d / 2
            for a in range(len(Xm[n])):
                e = Xm[n][a] - Xm[n - 1][a] - h * (F[n][a] + F[n - 1][a])
                A_d += mpf(float(spec.Rd[a])) * e * e / 2
        A = A_o + mpf(float(spec.beta)) * A_d
        return float(A), float(A_o), float(A_d)
