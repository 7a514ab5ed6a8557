"""Pins of the initialization phase (Section 4.2) in the oracle sampler.

* Annealing: beta starts at beta0, grows by f_beta = (1/beta0)^(1/N_cool)
  (eq. fbeta) after every sweep and is capped at 1, so it equals the closed
  form beta0 f_beta^k until sweep N_cool and 1 from there on.
* With beta0 = 1 and no step adjustment the phase is the plain sampler, bit
  for bit; with beta < 1 a sweep is the plain sweep of the model whose
  dynamical term carries that multiplier (the same random numbers).
* The step-size rule moves each step until the acceptance of its component
  is f_acc: its fixed point (checked statistically on the linear-Gaussian
  window, for the per-site state steps and for the parameter's step), and
  steps stay frozen after N_init.
"""

import numpy as np

import workloads as W
from oracle import sampler as OS


def test_beta_schedule_closed_form():
    st = OS.InitPhase(beta0=0.01, n_cool=50, n_init=0, n_skip=10).start(4, np.ones(1))
    L = W.make_lin1_problem(M=4)
    X, p = L.X0.copy(), L.p0.copy()
    betas = []
    for k in range(80):
        betas.append(st.beta)
        OS.run(L.model, X, p, L.y, L.I, seed=1, chain=0, sweep0=k, n_sweeps=1, w_state=L.w_state,
               w_param=L.w_param, flags=OS.STATES, init=st)
    betas = np.array(betas)
    k = np.arange(80)
    closed = np.minimum(1.0, 0.01 * (1.0 / 0.01) ** (k / 50.0))
    np.testing.assert_allclose(betas[:50], closed[:50], rtol=1e-12)
    assert abs(betas[50] - 1.0) < 1e-12 and (betas[51:] == 1.0).all()
    assert (np.diff(betas) >= 0).all()


def test_unit_phase_is_the_plain_sampler():
    prob = W.make_hh_problem(40, 0.02, 101, require_spike=False)
    X1, p1 = prob.X0.copy(), prob.p0.copy()
    X2, p2 = prob.X0.copy(), prob.p0.copy()
    kw = dict(seed=prob.seed, chain=1, sweep0=3, n_sweeps=6, w_state=prob.w_state, w_param=prob.w_param)
    OS.run(prob.model, X1, p1, prob.y, prob.I, **kw)
    st = OS.InitPhase(beta0=1.0, n_cool=1, n_init=0, n_skip=1).start(prob.M, prob.w_param)
    OS.run(prob.model, X2, p2, prob.y, prob.I, init=st, **kw)
    np.testing.assert_array_equal(X1, X2)
    np.testing.assert_array_equal(p1, p2)


def test_annealed_sweep_is_the_sweep_of_the_tempered_action():
    prob = W.make_hh_problem(40, 0.02, 102, require_spike=False)
    st = OS.InitPhase(beta0=0.05, n_cool=10, n_init=0, n_skip=1).start(prob.M, prob.w_param)
    X1, p1 = prob.X0.copy(), prob.p0.copy()
    OS.run(prob.model, X1, p1, prob.y, prob.I, seed=4, chain=0, sweep0=0, n_sweeps=1, w_state=prob.w_state,
           w_param=prob.w_param, init=st)
    X2, p2 = prob.X0.copy(), prob.p0.copy()
    OS.run(prob.model.with_(beta=0.05), X2, p2, prob.y, prob.I, seed=4, chain=0, sweep0=0, n_sweeps=1,
           w_state=prob.w_state, w_param=prob.w_param)
    np.testing.assert_array_equal(X1, X2)
    np.testing.assert_array_equal(p1, p2)
    assert not np.array_equal(X1, prob.X0)


def test_step_rule_reaches_target_acceptance_and_freezes():
    """On the linear-Gaussian window, starting from steps far too small (all
    proposals accepted), the rule drives every component's acceptance to
    f_acc = 0.23 (its fixed point); after N_init the steps no longer change."""
    L = W.make_lin1_problem(M=8, w=0.02)
    spec = L.model.with_(p_mask=1, p_lo=(0.01,), p_hi=(5.0,))
    X, p = L.X0.copy(), L.p0.copy()
    n_init, n_skip, n_post = 9000, 100, 5000
    st = OS.InitPhase(beta0=1.0, n_cool=1, n_init=n_init, n_skip=n_skip, f_acc=0.23, alpha=0.3).start(
        L.M, np.array([0.02]))
    OS.run(spec, X, p, L.y, L.I, seed=11, chain=0, sweep0=0, n_sweeps=n_init, w_state=L.w_state,
           w_param=L.w_param, init=st)
    scale = st.site_scale.copy()
    wpar = st.w_param.copy()
    OS.run(spec, X, p, L.y, L.I, seed=11, chain=0, sweep0=n_init, n_sweeps=n_post, w_state=L.w_state,
           w_param=L.w_param, init=st)
    np.testing.assert_array_equal(st.site_scale, scale)    # frozen after N_init
    np.testing.assert_array_equal(st.w_param, wpar)
    acc_sites = st.cnt_site / n_post
    assert abs(acc_sites.mean() - 0.23) < 0.015, acc_sites
    assert np.abs(acc_sites - 0.23).max() < 0.04, acc_sites
    # one component with its own count: its step keeps a random walk of a
    # few per cent about the fixed point (alpha = 0.3, 100-sweep counts)
    assert abs(st.cnt_param[0] / n_post - 0.23) < 0.05, st.cnt_param
    assert scale.min() > 5.0 and wpar[0] > 0.2      # both grew from steps far too small
