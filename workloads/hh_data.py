"""Synthetic Hodgkin-Huxley twin-experiment data (Section 5.1 stand-in).

Recipe (all FP64, all seeded):

* drive I(t) = 10 * [t >= t_on] + 5 sin(2 pi t / 10 ms) + eta(t), eta an
  Ornstein-Uhlenbeck process with tau = 1 ms and stationary sd 1 uA/cm^2,
  sampled exactly on the grid as an AR(1) recursion;
* truth: the HH equations (dV/dt and da/dt of Section 5.1, gating constants
  of Table 1) integrated with classical RK4, 10 sub-steps per dt, the drive
  linearly interpolated between grid points; the state at t=0 is the state
  after 50 ms at I = 0 starting from V = 0 with gates at their steady state;
* observations y_n = V(t_n) + N(0, sigma_obs^2), n = 1..M (only V is
  observed, L = 1);
* initial guess for the sampler: V_n = y_n (V_0 = y_1), gates at their
  steady-state value for that V, parameters uniform in the box.

The vector field below is this module's own copy: it exists to make data,
and shares no code with the sampler or with its checker.
"""

from __future__ import annotations

import math

import numpy as np

from .problem import GATES_MHN, P_STAR, ModelSpec, Problem


def _gate_inf_tau(V, g):
    Va, dVa, t0, t1 = g
    th = np.tanh((V - Va) / dVa)
    return 0.5 + 0.5 * th, t0 + t1 * (1.0 - th * th)


def _make_rhs(p, gates):
    """Scalar HH vector field (dV/dt and da/dt of Section 5.1) as a closure."""
    p1, p2, p3, p4, p5, p6, p7 = (float(v) for v in p)
    (Vm, dVm, t0m, t1m), (Vh, dVh, t0h, t1h), (Vn, dVn, t0n, t1n) = gates
    tanh = math.tanh

    def rhs(V, m, h, n, I):
        dV = p1 * I + p2 * m * m * m * h * (p3 - V) + p4 * n * n * n * n * (p5 - V) + p6 * (p7 - V)
        tm = tanh((V - Vm) / dVm)
        th = tanh((V - Vh) / dVh)
        tn = tanh((V - Vn) / dVn)
        dm = (0.5 + 0.5 * tm - m) / (t0m + t1m * (1.0 - tm * tm))
        dh = (0.5 + 0.5 * th - h) / (t0h + t1h * (1.0 - th * th))
        dn = (0.5 + 0.5 * tn - n) / (t0n + t1n * (1.0 - tn * tn))
        return dV, dm, dh, dn

    return rhs


def hh_stimulus(M: int, dt: float, rng: np.random.Generator, t_on: float = 1.0,
                step: float = 10.0, amp: float = 5.0, period: float = 10.0,
                ou_tau: float = 1.0, ou_sd: float = 1.0) -> np.ndarray:
    """Drive I_n at t_n = n dt, n = 0..M (step + sine + exact-AR(1) OU)."""
    t = np.arange(M + 1) * dt
    a = np.exp(-dt / ou_tau)
    s = ou_sd * np.sqrt(1.0 - a * a)
    eta = np.empty(M + 1)
    eta[0] = ou_sd * rng.standard_normal()
    xi = rng.standard_normal(M)
    for k in range(M):
        eta[k + 1] = a * eta[k] + s * xi[k]
    return step * (t >= t_on) + amp * np.sin(2.0 * np.pi * t / period) + eta


def _rk4(rhs, x, I0, I1, dt, sub):
    """Classical RK4 over one grid step with `sub` sub-steps; I linear in t."""
    V, m, h, n = x
    hs = dt / sub
    for j in range(sub):
        Ia = I0 + (I1 - I0) * (j / sub)
        Ib = I0 + (I1 - I0) * ((j + 0.5) / sub)
        Ic = I0 + (I1 - I0) * ((j + 1.0) / sub)
        a1 = rhs(V, m, h, n, Ia)
        a2 = rhs(V + 0.5 * hs * a1[0], m + 0.5 * hs * a1[1], h + 0.5 * hs * a1[2], n + 0.5 * hs * a1[3], Ib)
        a3 = rhs(V + 0.5 * hs * a2[0], m + 0.5 * hs * a2[1], h + 0.5 * hs * a2[2], n + 0.5 * hs * a2[3], Ib)
        a4 = rhs(V + hs * a3[0], m + hs * a3[1], h + hs * a3[2], n + hs * a3[3], Ic)
        c = hs / 6.0
        V = V + c * (a1[0] + 2 * a2[0] + 2 * a3[0] + a4[0])
        m = m + c * (a1[1] + 2 * a2[1] + 2 * a3[1] + a4[1])
        h = h + c * (a1[2] + 2 * a2[2] + 2 * a3[2] + a4[2])
        n = n + c * (a1[3] + 2 * a2[3] + 2 * a3[3] + a4[3])
    return (V, m, h, n)


def hh_rest_state(p=P_STAR, gates=GATES_MHN, settle_ms: float = 50.0, dt: float = 0.01):
    """State after `settle_ms` at I=0, from V=0 and gates at steady state."""
    rhs = _make_rhs(p, gates)
    x = (0.0,) + tuple(float(_gate_inf_tau(0.0, g)[0]) for g in gates)
    for _ in range(int(round(settle_ms / dt))):
        x = _rk4(rhs, x, 0.0, 0.0, dt, 1)
    return np.array(x)


def hh_truth(I: np.ndarray, dt: float, p=P_STAR, gates=GATES_MHN, sub: int = 10) -> np.ndarray:
    """RK4 trajectory on the grid, shape (M+1, 4)."""
    M = len(I) - 1
    rhs = _make_rhs(p, gates)
    X = np.empty((M + 1, 4))
    X[0] = hh_rest_state(p, gates)
    x = tuple(float(v) for v in X[0])
    Il = [float(v) for v in I]
    for k in range(M):
        x = _rk4(rhs, x, Il[k], Il[k + 1], dt, sub)
        X[k + 1] = x
    return X


def make_hh_problem(M: int, dt: float = 0.02, data_seed: int = 101, *,
                    model: ModelSpec | None = None, p_true=P_STAR,
                    sigma_obs: float = 1.0, t_on: float = 1.0,
                    w_state=(0.05, 5e-4, 5e-4, 5e-4), w_param_rel: float = 1e-3,
                    init: str = "guess", sampler_seed: int = 1, chain: int = 0,
                    require_spike: bool = True) -> Problem:
    """Build one HH window.

    init = "guess": the initial path of the recipe above (V from the data,
    gates at steady state, p uniform in the box); init = "truth": start at the
    true path and parameters (useful for short statistical checks).
    """
    model = model or ModelSpec(dt=dt)
    if model.dt != dt:
        model = model.with_(dt=dt)
    rng = np.random.default_rng(data_seed)
    I = hh_stimulus(M, dt, rng, t_on=t_on)
    p_true = np.asarray(p_true, dtype=np.float64)
    X = hh_truth(I, dt, p_true, model.gates)
    if require_spike and not (X[:, 0] > 50.0).any():
        raise ValueError("window holds no spike (V > 50 mV); move the step onset earlier")
    y = np.zeros(M + 1)
    y[1:] = X[1:, 0] + sigma_obs * rng.standard_normal(M)
    lo = np.asarray(model.p_lo)
    hi = np.asarray(model.p_hi)
    if init == "truth":
        X0 = X.copy()
        p0 = p_true.copy()
    else:
        X0 = np.empty_like(X)
        X0[1:, 0] = y[1:]
        X0[0, 0] = y[1]
        for j, g in enumerate(model.gates):
            X0[:, 1 + j] = _gate_inf_tau(X0[:, 0], g)[0]
        p0 = lo + (hi - lo) * rng.random(7)
    xlo = np.asarray(model.x_lo)
    xhi = np.asarray(model.x_hi)
    X0 = np.clip(X0, xlo, xhi)
    w_param = w_param_rel * np.abs(np.asarray(P_STAR))
    return Problem(model=model, M=M, y=y, I=I, X0=X0, p0=p0,
                   w_state=np.asarray(w_state, dtype=np.float64),
                   w_param=np.asarray(w_param, dtype=np.float64),
                   seed=sampler_seed, chain=chain, X_true=X, p_true=p_true,
                   meta={"data_seed": data_seed, "sigma_obs": sigma_obs, "t_on": t_on})
