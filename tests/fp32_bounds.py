"""First-order rounding bounds for the FP32 site arithmetic (test support).

The FP32 kernels evaluate the HH field, the link errors eps_n and the action
gradient in single precision from FP32 inputs.  These helpers bound, element
by element, how far such a result may lie from the FP64 oracle's value on the
same (FP32-representable) inputs: every rounded operation contributes at most
u = 2^-24 times the magnitude of what it produces, and the hardware tanh
(exp2 and reciprocal, each within a few ulp) contributes an absolute error
of at most TANH_ABS.  Errors are propagated to first order through the
formulas of Section 2.1 (trapezoid link error, local gradient stencil), with
magnitudes taken from the oracle's own intermediate values.  A factor SAFETY
covers the few extra roundings per formula that the counts below fold in.
"""

from __future__ import annotations

import numpy as np

from oracle.models import model_for

U = 2.0 ** -24
TANH_ABS = 8.0 * U
SAFETY = 4.0


def _field_parts(spec, X, I, p):
    """F, dF bound (per site and component), J and dJ bound of the HH field."""
    X = np.asarray(X, dtype=np.float64)
    I = np.asarray(I, dtype=np.float64)
    V, m, h, n = X[:, 0], X[:, 1], X[:, 2], X[:, 3]
    mod = model_for(spec)
    F = mod.F(X, I, p)
    J = mod.J(X, p)
    m3h = m ** 3 * h
    n4 = n ** 4
    N = X.shape[0]
    dF = np.zeros((N, 4))
    dJ = np.zeros((N, 4, 4))
    # dV/dt: a sum of four products, each formed with a handful of roundings;
    # p and the inputs are themselves rounded to FP32 on the device
    sV = (np.abs(p[0] * I) + abs(p[1]) * m3h * (abs(p[2]) + np.abs(V)) + abs(p[3]) * n4 * (abs(p[4]) + np.abs(V))
          + abs(p[5]) * (abs(p[6]) + np.abs(V)))
    dF[:, 0] = 8.0 * U * sV
    dJ[:, 0, 0] = 8.0 * U * (abs(p[1]) * m3h + abs(p[3]) * n4 + abs(p[5]))
    dJ[:, 0, 1] = 8.0 * U * 3.0 * abs(p[1]) * m ** 2 * h * (abs(p[2]) + np.abs(V))
    dJ[:, 0, 2] = 8.0 * U * abs(p[1]) * m ** 3 * (abs(p[2]) + np.abs(V))
    dJ[:, 0, 3] = 8.0 * U * 4.0 * abs(p[3]) * n ** 3 * (abs(p[4]) + np.abs(V))
    for j in range(3):
        Va, dVa, t0, t1 = spec.gates[j]
        a = X[:, 1 + j]
        s = (V - Va) / dVa
        t = np.tanh(s)
        sech2 = 1.0 - t * t
        ainf = 0.5 + 0.5 * t
        tau = t0 + t1 * sech2
        # tanh of the FP32 argument: the argument's own rounding moves t by
        # sech2 * |s| * 3u; the hardware evaluation adds TANH_ABS
        dt_ = sech2 * np.abs(s) * 3.0 * U + TANH_ABS
        dtau = abs(t1) * 2.0 * np.abs(t) * dt_ + 4.0 * U * tau
        dainf = 0.5 * dt_ + U
        dF[:, 1 + j] = (dainf + 2.0 * U * (np.abs(ainf) + np.abs(a))) / tau + np.abs(F[:, 1 + j]) * (dtau / tau + 2 * U)
        term1 = np.abs(0.5 * sech2 / dVa / tau)
        term2 = np.abs((ainf - a) * 2.0 * t1 * t * sech2 / dVa / tau ** 2)
        dJ[:, 1 + j, 0] = 16.0 * U * (term1 + term2) + dt_ * (1.0 + 2.0 * abs(t1) / tau) * 3.0 / (abs(dVa) * tau) \
            + (term1 + term2) * 2.0 * dtau / tau
        dJ[:, 1 + j, 1 + j] = np.abs(J[:, 1 + j, 1 + j]) * (dtau / tau + 2 * U)
    return F, dF, J, dJ


def link_bounds(spec, X, I, p):
    """v = beta Rd eps for links n = 1..M (shape (M, 4)) and its FP32 error bound."""
    X = np.asarray(X, dtype=np.float64)
    F, dF, J, dJ = _field_parts(spec, X, I, p)
    hs = 0.5 * spec.dt
    dx = X[1:] - X[:-1]
    e = dx - hs * (F[1:] + F[:-1])
    de = (2.0 * U * (np.abs(dx) + 2.0 * hs * (np.abs(F[1:]) + np.abs(F[:-1])) + np.abs(e))
          + hs * (dF[1:] + dF[:-1]))
    bR = spec.beta * np.asarray(spec.Rd, dtype=np.float64)[None, :]
    v = bR * e
    dv = bR * de + 2.0 * U * np.abs(v)
    return v, dv, F, dF, J, dJ


def grad_bound(spec, X, y, I, p):
    """Element-wise bounds of |g_FP32 - g_FP64| for dA/dX (M+1, 4) and dA/dp (7,)."""
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    M = X.shape[0] - 1
    v, dv, F, dF, J, dJ = link_bounds(spec, X, I, p)
    hs = 0.5 * spec.dt
    vl = np.zeros((M + 1, 4))
    vr = np.zeros((M + 1, 4))
    dvl = np.zeros((M + 1, 4))
    dvr = np.zeros((M + 1, 4))
    vl[1:], dvl[1:] = v, dv          # link n (n >= 1) ends at site n
    vr[:-1], dvr[:-1] = v, dv        # link n + 1 starts at site n
    w = vl + vr
    dw = dvl + dvr
    uu = vl - vr
    # g_a = u_a - h sum_c J_ca w_c  (J[c, a] = dF_c / dx_a)
    Jt = np.abs(J)
    jw = np.einsum("nca,nc->na", Jt, np.abs(w))
    bound = (dvl + dvr + hs * (np.einsum("nca,nc->na", Jt, dw) + np.einsum("nca,nc->na", dJ, np.abs(w)))
             + 4.0 * U * (np.abs(vl) + np.abs(vr) + hs * jw))
    bound[1:, 0] += 2.0 * U * spec.Ro * (np.abs(y[1:]) + np.abs(X[1:, 0]) + np.abs(y[1:] - X[1:, 0]))
    # dA/dp: per link -h v_V (dF_V/dp at both ends), the dF_V/dp factors in FP64
    mod = model_for(spec)
    dFp = mod.dF_dp(X, np.asarray(I, dtype=np.float64), p)[:, 0, :]     # (M+1, 7)
    s = np.abs(dFp[1:]) + np.abs(dFp[:-1])
    gp_bound = hs * (dv[:, 0][:, None] * s).sum(axis=0) + 1e-12 * hs * (np.abs(v[:, 0])[:, None] * s).sum(axis=0)
    return SAFETY * bound, SAFETY * gp_bound


def box_muller_bound(block):
    """Bound of |z_FP32 - z_FP64| for the four normals of each Philox block
    (rows of `block`, words (0, 1) and (2, 3) paired as in the generator
    contract) when the radius and angle are formed in FP32: u_a is rounded
    to FP32 (half an ulp, at most 2^-25 absolute below 1), the hardware
    logarithm adds a few ulp of its result, so r^2 = -2 ln u_a carries an
    absolute error e2 and r an error min(e2 / r, sqrt(e2)) (the square root
    near u_a = 1 amplifies it); the angle carries a few ulp of a revolution."""
    block = np.asarray(block, dtype=np.float64)
    out = np.empty(block.shape)
    for j in (0, 2):
        ua = (block[:, j] + 0.5) * 2.0 ** -32
        r = np.sqrt(-2.0 * np.log(ua))
        e2 = 2.0 * (2.0 ** -25 / ua + 4.0 * U * np.abs(np.log(ua))) + 8.0 * U * r * r
        dr = np.minimum(e2 / np.maximum(r, 1e-300), np.sqrt(e2))
        dz = 2.0 * dr + r * (2.0 * np.pi * 16.0 * U + 4.0 * U) + 1e-7
        out[:, j] = dz
        out[:, j + 1] = dz
    return SAFETY * out
