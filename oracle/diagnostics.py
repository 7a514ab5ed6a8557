"""Model checks of Section 6 (oracle, FP64).

* Model and observation errors of a path: eps_n (Section 2.1, trapezoid
  rule) and delta_n = y_n - V_n for n = 1..M.  If the model is right, their
  means over the posterior are zero and their variances are 1/Rd and 1/Ro
  (Section 6); the discretisation shows up as <eps_n> away from zero where V
  spikes.
* Forecast: the model integrated forward from a final state x_M with
  parameters p, either once from the posterior means <x_M>, <p> or as an
  ensemble over posterior samples with model noise (Section 6).  Reading:
  the integrator is Heun's method (the explicit form of the trapezoid rule
  that defines the model error), and the noise of a step is the model error
  the action assumes, eps ~ N(0, 1/Rd) per component, times `noise`; its
  normals come from the Philox FCST block of (member, step).
"""

from __future__ import annotations

import numpy as np

from . import philox as ph
from .action import eps
from .models import model_for

TAG_FCST = 8


def model_errors(spec, X, y, I, p):
    """(eps (M, D), delta (M,)) of one path."""
    X = np.asarray(X, dtype=np.float64)
    e = eps(model_for(spec), X, np.asarray(I, dtype=np.float64), p, spec.dt)
    d = np.asarray(y, dtype=np.float64)[1:] - X[1:, 0]
    return e, d


def forecast(spec, x0, p, I, n, *, noise=0.0, seed=0, member=0):
    """Trajectory (n+1, D) from x0 over the drive I[0..n] (I[0] at x0's time)."""
    model = model_for(spec)
    dt = spec.dt
    sd = 1.0 / np.sqrt(np.asarray(spec.Rd, dtype=np.float64))
    out = np.empty((n + 1, len(x0)))
    x = np.asarray(x0, dtype=np.float64).copy()
    out[0] = x
    for k in range(n):
        k1 = model.F(x[None, :], np.array([I[k]]), p)[0]
        xt = x + dt * k1
        k2 = model.F(xt[None, :], np.array([I[k + 1]]), p)[0]
        x = x + 0.5 * dt * (k1 + k2)
        if noise != 0.0:
            z = ph.normals4(ph.draw(seed, 0, member, k, TAG_FCST))[0][:len(x)]
            x = x + noise * sd * z
        out[k + 1] = x
    return out
