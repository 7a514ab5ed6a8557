"""Pins of the exact conditional parameter draw (oracle/gibbs.py).

The conditional density of p_l given the path and the other parameters is
exp(-A) restricted to p_l's box; A is evaluated here point by point on a
grid with the oracle's direct-sum parameter action change (itself pinned to
brute force in test_oracle_action), and the grid's quadrature moments are
compared with the moments of the oracle's draws taken at a regular grid of
uniforms (a Riemann sum of the quantile function, so no sampling noise):
a wrong mean, a wrong width, a wrong tail branch or a mistaken truncation
of the inverse-CDF draw fails these.
"""

import numpy as np
import pytest

import workloads as W
from oracle import gibbs as OG
from oracle import sampler as OS
from oracle.action import delta_params


def _grid_moments(spec, X, I, p, l, n=20001):
    """Mean and variance of exp(-A) over p_l's box by quadrature; a second,
    finer grid around the mass when the coarse one under-resolves it."""
    lo, hi = spec.p_lo[l], spec.p_hi[l]

    def moments(a, b):
        v = np.linspace(a, b, n)
        dA = np.empty(n)
        for i, vi in enumerate(v):
            q = p.copy()
            q[l] = vi
            dA[i] = delta_params(spec, X, I, p, q)
        w = np.exp(-(dA - dA.min()))
        w[0] *= 0.5
        w[-1] *= 0.5
        m = (w * v).sum() / w.sum()
        return m, (w * (v - m) ** 2).sum() / w.sum()

    m, var = moments(lo, hi)
    sd = np.sqrt(var)
    if sd < 200 * (hi - lo) / n:
        m, var = moments(max(lo, m - 14 * sd), min(hi, m + 14 * sd))
    return m, var


def _draw_moments(spec, X, I, p, l, n=200001):
    mu, sigma = OG.conditional(spec, X, I, p, l)
    u = (np.arange(n) + 0.5) / n
    v = np.asarray(OG.truncnorm_inverse(mu, sigma, spec.p_lo[l], spec.p_hi[l], u), dtype=np.float64)
    assert (v >= spec.p_lo[l]).all() and (v <= spec.p_hi[l]).all()
    return v.mean(), v.var()


def _window(M=30, seed=101):
    spec = W.ModelSpec(p_mask=0x7F)
    prob = W.make_hh_problem(M, 0.02, seed, model=spec, require_spike=False, init="truth")
    return prob


@pytest.mark.parametrize("l", range(7))
def test_conditional_draw_matches_quadrature(l):
    prob = _window()
    X = prob.X_true
    p = np.asarray(prob.p_true) * 1.03
    m_q, v_q = _grid_moments(prob.model, X, prob.I, p, l)
    m_d, v_d = _draw_moments(prob.model, X, prob.I, p, l)
    sd = np.sqrt(v_q)
    assert abs(m_d - m_q) < 2e-3 * sd, (m_d, m_q, sd)
    assert abs(v_d / v_q - 1.0) < 5e-3


@pytest.mark.parametrize("side", ["below", "above"])
def test_truncated_conditional_matches_quadrature(side):
    """A box that cuts the Gaussian (its mean outside the box, on either
    side): the draws follow the truncated density, tails included."""
    prob = _window(M=24, seed=107)
    X = prob.X_true
    p = np.asarray(prob.p_true, dtype=np.float64)
    l = 5                                   # g_L
    mu, sigma = OG.conditional(prob.model, X, prob.I, p, l)
    assert np.isfinite(sigma)
    if side == "below":                     # box entirely above the mean, 2..6 sd away
        lo, hi = mu + 2 * sigma, mu + 6 * sigma
    else:
        lo, hi = mu - 6 * sigma, mu - 2 * sigma
    p_lo = list(prob.model.p_lo)
    p_hi = list(prob.model.p_hi)
    p_lo[l], p_hi[l] = lo, hi
    spec = prob.model.with_(p_lo=tuple(p_lo), p_hi=tuple(p_hi))
    p[l] = 0.5 * (lo + hi)
    m_q, v_q = _grid_moments(spec, X, prob.I, p, l)
    m_d, v_d = _draw_moments(spec, X, prob.I, p, l)
    sd = np.sqrt(v_q)
    assert abs(m_d - m_q) < 2e-3 * sd
    assert abs(v_d / v_q - 1.0) < 5e-3


@pytest.mark.parametrize("dist", [8.0, 45.0])
def test_far_tail_box_draws_stay_in_the_box_and_follow_the_tail(dist):
    """A path far from the data can put the conditional mean many standard
    deviations below the box: every draw is finite, inside the box, and
    follows the truncated density (the mean of Z given Z > a is the inverse
    Mills ratio phi(a) / Q(a), the box's far end adding nothing visible)."""
    from scipy.special import erfcx
    mu, sigma = 0.0, 1.0
    lo, hi = dist, dist + 10.0
    u = (np.arange(20001) + 0.5) / 20001
    v = np.asarray(OG.truncnorm_inverse(mu, sigma, lo, hi, u), dtype=np.float64)
    assert np.isfinite(v).all() and (v >= lo).all() and (v <= hi).all()
    m = v.mean()
    mills = np.sqrt(2.0 / np.pi) / erfcx(dist / np.sqrt(2.0))
    assert abs(m - mills) < 1e-5


def test_gibbs_sweep_uses_the_parameter_stream_and_keeps_the_path():
    """A Gibbs parameter sweep moves every sampled parameter inside its box,
    leaves the path alone and depends only on (seed, chain, sweep)."""
    prob = _window()
    X = prob.X_true.copy()
    p1 = np.asarray(prob.p0, dtype=np.float64).copy()
    p2 = p1.copy()
    OS.run(prob.model, X, p1, prob.y, prob.I, seed=5, chain=2, sweep0=9, n_sweeps=1, w_state=prob.w_state,
           w_param=prob.w_param, flags=OS.PARAMS | OS.GIBBS)
    OS.run(prob.model, X.copy(), p2, prob.y, prob.I, seed=5, chain=2, sweep0=9, n_sweeps=1,
           w_state=prob.w_state, w_param=prob.w_param * 3.0, flags=OS.PARAMS | OS.GIBBS)
    np.testing.assert_array_equal(X, prob.X_true)
    np.testing.assert_array_equal(p1, p2)       # widths play no part in a Gibbs draw
    assert ((p1 >= prob.model.p_lo) & (p1 <= prob.model.p_hi)).all()
    assert (p1 != prob.p0).all()
