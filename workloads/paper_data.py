"""The paper-like twin experiment of Section 5.1 (stand-in for its data).

The paper drives its HH neuron with a chaotic current taken from one
variable of the Lorenz system and samples V at 25 kHz (dt = 0.04 ms,
M = 8000, 320 ms); its data are not available.  This recipe builds data of
that structure:

* Lorenz system (sigma, rho, b) = (10, 28, 8/3) integrated with RK4 (step
  1e-3 Lorenz time units) from a seeded point near the attractor after a
  discarded transient; one Lorenz time unit spans `tau_ms` = 8 ms of neuron
  time, and I(t) = I0 + c * x_L(t / tau_ms) with I0 = 6 and c = 0.4 uA/cm^2
  (readings: the paper gives neither the scale of the current nor its time
  scale; these values make the neuron spike irregularly, as in its Fig. 3);
* truth: the same RK4 integration of the HH equations as the other
  workloads (hh_data), continued `n_future` steps beyond the window for the
  forecast check of Section 6;
* y_n = V(t_n) + N(0, 1/Ro), Ro = 100 as in Section 5.1 (well specified);
* model: Rd = (100, 1e6, 1e6, 1e6), seven parameters sampled, uniform
  proposals of Fig. 1 with initial steps 2e-3 (V), 1e-3 (gates) and
  1e-3 |p*| (parameters), as in Section 5.1.
"""

from __future__ import annotations

import numpy as np

from .hh_data import _gate_inf_tau, hh_truth
from .problem import P_STAR, ModelSpec, Problem

PAPER_RUN = dict(M=8000, dt=0.04, Ro=100.0, sweeps=1_000_000, n_skip=400, n_init=500_000, n_cool=100_000,
                 beta0=0.01, f_acc=0.23, alpha=0.02)


def lorenz_drive(n: int, dt_ms: float, seed: int, tau_ms: float = 8.0, I0: float = 6.0, c: float = 0.4):
    """I_n at t_n = n dt_ms, n = 0..n-1, from the x variable of Lorenz-63."""
    rng = np.random.default_rng(seed)
    s, r, b = 10.0, 28.0, 8.0 / 3.0

    def f(v):
        x, y, z = v
        return np.array([s * (y - x), x * (r - z) - y, x * y - b * z])

    h = 1e-3
    v = np.array([1.0, 1.0, 20.0]) + rng.standard_normal(3)
    for _ in range(20000):                       # transient onto the attractor
        k1 = f(v); k2 = f(v + 0.5 * h * k1); k3 = f(v + 0.5 * h * k2); k4 = f(v + h * k3)
        v = v + h / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
    # sample x at the neuron grid: neuron step dt_ms = dt_ms / tau_ms Lorenz units
    per = dt_ms / tau_ms
    sub = max(1, int(np.ceil(per / h)))
    hh = per / sub
    out = np.empty(n)
    for i in range(n):
        out[i] = v[0]
        for _ in range(sub):
            k1 = f(v); k2 = f(v + 0.5 * hh * k1); k3 = f(v + 0.5 * hh * k2); k4 = f(v + hh * k3)
            v = v + hh / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
    return I0 + c * out


def make_paper_problem(M: int = 8000, dt: float = 0.04, Ro: float = 100.0, data_seed: int = 2011,
                       n_future: int = 1000, p_true=P_STAR, sampler_seed: int = 7) -> Problem:
    """The paper-like window plus its continuation (meta: I_future, X_future,
    y_future over n_future further steps)."""
    model = ModelSpec(dt=dt, Ro=Ro, proposal="uniform", p_mask=0x7F)
    rng = np.random.default_rng(data_seed)
    I_all = lorenz_drive(M + 1 + n_future, dt, data_seed + 1)
    p_true = np.asarray(p_true, dtype=np.float64)
    X_all = hh_truth(I_all, dt, p_true, model.gates)
    y_all = X_all[:, 0] + rng.standard_normal(len(X_all)) / np.sqrt(Ro)
    y = y_all[:M + 1].copy()
    y[0] = 0.0
    I = I_all[:M + 1].copy()
    X = X_all[:M + 1].copy()
    lo, hi = np.asarray(model.p_lo), np.asarray(model.p_hi)
    X0 = np.empty_like(X)
    X0[1:, 0] = y[1:]
    X0[0, 0] = y[1]
    for j, g in enumerate(model.gates):
        X0[:, 1 + j] = _gate_inf_tau(X0[:, 0], g)[0]
    X0 = np.clip(X0, np.asarray(model.x_lo), np.asarray(model.x_hi))
    p0 = lo + (hi - lo) * rng.random(7)
    return Problem(model=model, M=M, y=y, I=I, X0=X0, p0=p0,
                   w_state=np.array([2e-3, 1e-3, 1e-3, 1e-3]), w_param=1e-3 * np.abs(np.asarray(P_STAR)),
                   seed=sampler_seed, chain=0, X_true=X, p_true=p_true,
                   meta={"data_seed": data_seed, "I_future": I_all[M:], "X_future": X_all[M:],
                         "y_future": y_all[M:], "spikes": int(((X[1:, 0] > 50) & (X[:-1, 0] <= 50)).sum())})
