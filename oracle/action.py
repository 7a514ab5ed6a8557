"""Action, local action change and gradient (oracle, FP64).

Section 2.1 of the paper: with the observation error delta_n = y_n - h(x_n)
(h(x) = V, L = 1) and the trapezoid model error

    eps_n = x_n - x_{n-1} - (dt/2) [F(x_n) + F(x_{n-1})],     n = 1..M,

the action is A = A_o + beta * A_d with
    A_o = 1/2 sum_{n=1..M} Ro delta_n^2,
    A_d = 1/2 sum_{n=1..M} eps_n^T Rd eps_n          (Rd diagonal),
where beta is the annealing multiplier of the dynamical term (Section 4.2).
The uniform box prior contributes a constant inside the box and is handled by
rejection, never by evaluating A outside it.
"""

from __future__ import annotations

import math

import numpy as np

from .models import model_for


def eps(model, X, I, p, dt):
    """Model errors eps_1..eps_M, shape (M, D)."""
    F = model.F(X, I, p)
    return X[1:] - X[:-1] - 0.5 * dt * (F[1:] + F[:-1])


def action(spec, X, y, I, p):
    """(A, A_o, A_d) with A = A_o + beta * A_d, each summed exactly (fsum)."""
    X = np.asarray(X, dtype=np.float64)
    model = model_for(spec)
    e = eps(model, X, I, p, spec.dt)
    Rd = np.asarray(spec.Rd, dtype=np.float64)
    d = np.asarray(y[1:], dtype=np.float64) - X[1:, 0]
    A_o = 0.5 * math.fsum((spec.Ro * d * d).tolist())
    A_d = 0.5 * math.fsum((Rd[None, :] * e * e).ravel().tolist())
    return spec.beta * A_d + A_o, A_o, A_d


def delta_site(spec, X, y, I, p, ns, xprop):
    """A(X') - A(X) when x_n is replaced by xprop (one row per n in ns).

    Only the terms that contain x_n change (Section 3.1: only the changed
    terms need computing): the observation term at n (n >= 1) and the model
    errors of the links (n-1, n) (n >= 1) and (n, n+1) (n <= M-1).  Each
    changed term is evaluated old and new in full and subtracted.
    """
    X = np.asarray(X, dtype=np.float64)
    model = model_for(spec)
    M = X.shape[0] - 1
    ns = np.asarray(ns, dtype=np.int64)
    xprop = np.asarray(xprop, dtype=np.float64).reshape(len(ns), -1)
    Rd = np.asarray(spec.Rd, dtype=np.float64)
    h = 0.5 * spec.dt
    nm = np.clip(ns - 1, 0, M)
    npl = np.clip(ns + 1, 0, M)
    xm, x0, xpl = X[nm], X[ns], X[npl]
    Fm = model.F(xm, I[nm], p)
    F0 = model.F(x0, I[ns], p)
    Fn = model.F(xprop, I[ns], p)
    Fp = model.F(xpl, I[npl], p)
    # link (n-1, n)
    e_old = x0 - xm - h * (F0 + Fm)
    e_new = xprop - xm - h * (Fn + Fm)
    dyn = ((e_new * e_new - e_old * e_old) * Rd).sum(axis=1) * (ns >= 1)
    # link (n, n+1)
    f_old = xpl - x0 - h * (Fp + F0)
    f_new = xpl - xprop - h * (Fp + Fn)
    dyn = dyn + ((f_new * f_new - f_old * f_old) * Rd).sum(axis=1) * (ns <= M - 1)
    yn = np.asarray(y, dtype=np.float64)[ns]
    obs = ((yn - xprop[:, 0]) ** 2 - (yn - x0[:, 0]) ** 2) * (ns >= 1)
    return 0.5 * spec.beta * dyn + 0.5 * spec.Ro * obs


def delta_params(spec, X, I, p, pprop):
    """A(X, p') - A(X, p) by the direct sum over every link (Section 4.1).

    Only the dynamical term depends on p; its change is summed over all
    n = 1..M exactly (fsum), the way the paper's parameter kernel does it.
    """
    X = np.asarray(X, dtype=np.float64)
    model = model_for(spec)
    Rd = np.asarray(spec.Rd, dtype=np.float64)
    e0 = eps(model, X, I, p, spec.dt)
    e1 = eps(model, X, I, pprop, spec.dt)
    terms = (Rd[None, :] * (e1 * e1 - e0 * e0)).ravel()
    return 0.5 * spec.beta * math.fsum(terms.tolist())


def delta_kinetic(spec, X, I, p, gates_new):
    """A(X, p; gates') - A(X, p; gates) by the direct sum over every link.

    The gating constants of Table 1 enter only the gate equations of F
    (Section 5.1), so only the dynamical term changes; like the parameter
    moves of Section 4.1 the change is summed over all n = 1..M (fsum)."""
    X = np.asarray(X, dtype=np.float64)
    Rd = np.asarray(spec.Rd, dtype=np.float64)
    e0 = eps(model_for(spec), X, I, p, spec.dt)
    e1 = eps(model_for(spec.with_(gates=tuple(tuple(g) for g in gates_new))), X, I, p, spec.dt)
    terms = (Rd[None, :] * (e1 * e1 - e0 * e0)).ravel()
    return 0.5 * spec.beta * math.fsum(terms.tolist())


def grad(spec, X, y, I, p):
    """Analytic gradient (dA/dX (M+1, D), dA/dp (Np,)).

    A is a sum of terms that each touch one link or one site, so dA/dx_n is a
    local stencil:
      dA/dx_n = beta (1 - h J_n)^T Rd eps_n     [n >= 1]
              + beta (-1 - h J_n)^T Rd eps_{n+1} [n <= M-1]
              - Ro (y_n - V_n) e_V               [n >= 1]
      dA/dp   = -beta h sum_n eps_n^T Rd [dF/dp(x_n) + dF/dp(x_{n-1})]
    with h = dt/2 and J = dF/dx.
    """
    X = np.asarray(X, dtype=np.float64)
    model = model_for(spec)
    h = 0.5 * spec.dt
    Rd = np.asarray(spec.Rd, dtype=np.float64)
    J = model.J(X, p)
    v = spec.beta * Rd[None, :] * eps(model, X, I, p, spec.dt)      # (M, D)
    g = np.zeros_like(X)
    g[1:] += v - h * np.einsum("nab,na->nb", J[1:], v)
    g[:-1] += -v - h * np.einsum("nab,na->nb", J[:-1], v)
    g[1:, 0] -= spec.Ro * (np.asarray(y[1:], dtype=np.float64) - X[1:, 0])
    dFp = model.dF_dp(X, I, p)                                        # (N, D, Np)
    gp = -h * np.einsum("na,nal->l", v, dFp[1:] + dFp[:-1])
    return g, gp
