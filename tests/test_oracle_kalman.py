"""The closed-form posterior of the linear-Gaussian window against a Kalman
filter with a Rauch-Tung-Striebel backward pass.

Both describe exp(-A) of the D=1 window dx/dt = -lam x + I (Section 2.1's
trapezoid model error, observation of x with precision Ro; Section 1: the
Kalman solution is exact here) with a N(0, v) prior on x_0: one solves the
tridiagonal precision system, the other runs the filter forward and the
smoother backward.  They share nothing but the model coefficients, so a
wrong sign or index in either the precision matrix or the right-hand side
(or in the filter) shows up as a disagreement.
"""

import numpy as np
import pytest

import workloads as W
from oracle import kalman as OK


@pytest.mark.parametrize("M,lam,prior_var,Ro", [(16, 0.5, 1e2, 4.0), (40, 1.3, 1e4, 0.5), (5, 0.1, 1.0, 25.0)])
def test_lin1_closed_form_equals_rts_smoother(M, lam, prior_var, Ro):
    L = W.make_lin1_problem(M=M, lam=lam, Ro=Ro, data_seed=11 + M)
    m1, v1 = OK.lin1_posterior(L.model, L.y, L.I, lam, prior_var=prior_var)
    m2, v2 = OK.rts_smoother(L.model, L.y, L.I, lam, prior_var=prior_var)
    np.testing.assert_allclose(m1, m2, rtol=1e-9, atol=1e-9 * np.abs(m1).max())
    np.testing.assert_allclose(v1, v2, rtol=1e-9)


def test_flat_prior_is_the_limit_of_wide_priors():
    """The sampler's flat prior on x_0 is the limit v -> inf of the smoother's."""
    L = W.make_lin1_problem(M=24, lam=0.7)
    m_flat, v_flat = OK.lin1_posterior(L.model, L.y, L.I, 0.7)
    # a prior of variance v moves the posterior by O(var_0 / v); much wider
    # priors cost the filter's forward variances their precision at n = 0
    m_wide, v_wide = OK.rts_smoother(L.model, L.y, L.I, 0.7, prior_var=1e6)
    np.testing.assert_allclose(m_flat, m_wide, rtol=1e-5, atol=1e-5)
    np.testing.assert_allclose(v_flat, v_wide, rtol=1e-5)


def test_smoother_marginal_variances_shrink_with_data():
    """Posterior variances lie below the prior and the observation variance
    wherever a site is observed (n >= 1), as conditioning on data requires."""
    L = W.make_lin1_problem(M=30, lam=0.5, Ro=4.0)
    _, v = OK.rts_smoother(L.model, L.y, L.I, 0.5, prior_var=1e2)
    assert (v[1:] < 1.0 / L.model.Ro).all()
    assert v[0] < 1e2
