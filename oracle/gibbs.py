"""Exact conditional draw of one parameter given the path (oracle, FP64).

The parameters enter the HH vector field only through dV/dt, and each p_l
enters it affinely when the others are held fixed (Section 5.1: dV/dt =
p1 I + p2 m^3 h (p3 - V) + p4 n^4 (p5 - V) + p6 (p7 - V)).  The model error
eps_{n,V} of Section 2.1 is then affine in p_l, so the action A(X, p) is a
quadratic polynomial in p_l and the conditional density of p_l given X and
the other parameters, exp(-A) on the box of p_l (the uniform prior of
Section 2.1), is a Gaussian truncated to that box.  Fig. 1 step 3 moves each
parameter in turn; drawing p_l from this conditional instead of proposing a
Metropolis step is the Gibbs form of the same step.

The oracle finds the quadratic by evaluating the change of A at three points
of the box with the direct sum over the path (Section 4.1), reads off the
mean and variance, and draws by inversion of the truncated normal CDF with
one uniform from the parameter's Philox block (word 0; word 2 stays the
Metropolis accept uniform); the inversion is SciPy's truncated-normal
quantile, which stays accurate when the box lies far out in a tail of the
Gaussian (a path far from the data makes the conditional mean of a
parameter sit many standard deviations outside its box).  A conditional
that is not a proper Gaussian (curvature not positive, or not finite) is
drawn uniformly on the box.
"""

from __future__ import annotations

import numpy as np
from scipy.stats import truncnorm

from . import philox as ph
from .action import delta_params


def conditional(spec, X, I, p, l):
    """(mu, sigma) of the Gaussian exp(-A) in p_l (unit: p_l), from the action
    at the box's two ends and centre; sigma = inf when the curvature is not
    positive."""
    lo, hi = float(spec.p_lo[l]), float(spec.p_hi[l])
    mid = 0.5 * (lo + hi)
    half = 0.5 * (hi - lo)
    d = []
    for v in (lo, mid, hi):
        q = np.array(p, dtype=np.float64)
        q[l] = v
        d.append(delta_params(spec, X, I, p, q))
    a = (d[0] + d[2] - 2.0 * d[1]) / (2.0 * half * half)     # A = a v^2 + ...
    slope = (d[2] - d[0]) / (2.0 * half)                     # dA/dv at mid
    if not (np.isfinite(a) and a > 0.0):
        return mid, np.inf
    return mid - slope / (2.0 * a), 1.0 / np.sqrt(2.0 * a)


def truncnorm_inverse(mu, sigma, lo, hi, u):
    """The u-quantile (u scalar or array) of N(mu, sigma^2) truncated to
    [lo, hi]."""
    if not np.isfinite(sigma):
        return lo + np.asarray(u) * (hi - lo)
    return truncnorm.ppf(u, (lo - mu) / sigma, (hi - mu) / sigma, loc=mu, scale=sigma)


def gibbs_draw_uniform(seed, chain, k, l):
    """The uniform of parameter l's Gibbs draw at sweep k: word 0 of its block."""
    b = ph.draw(seed, chain, l, k, ph.TAG_PARAM)[0]
    return float(ph.uniform_open(b[0]))


def param_gibbs(spec, X, I, p, k, seed, chain, acc=None, debug=None):
    """Each sampled parameter in ascending order drawn from its exact
    conditional given X and the current other parameters (in place on p).
    A draw that is not finite keeps p_l and is counted as non-finite."""
    lo_all, hi_all = np.asarray(spec.p_lo), np.asarray(spec.p_hi)
    for l in range(len(p)):
        if not (spec.p_mask >> l) & 1:
            continue
        mu, sigma = conditional(spec, X, I, p, l)
        u = gibbs_draw_uniform(seed, chain, k, l)
        v = float(truncnorm_inverse(mu, sigma, lo_all[l], hi_all[l], u))
        ok = bool(np.isfinite(v))
        if ok:
            v = min(max(v, lo_all[l]), hi_all[l])
            p[l] = v
            if acc is not None:
                acc[2 + l] += 1
        elif acc is not None:
            acc[9] += 1
        if debug is not None:
            debug.pprop[l] = v
            debug.pdA[l] = np.nan
            debug.pu[l] = u
            debug.paccept[l] = ok
