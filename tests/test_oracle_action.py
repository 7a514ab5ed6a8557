"""Pins of the oracle's action, local action change and gradient.

* A against a 50-digit mpmath evaluation on tiny windows (Section 2.1);
* the local dA of one site move equals the brute-force A(X') - A(X)
  (exactly summed) at every n, including the end sites 0 and M (Section 3.1);
* the direct-sum parameter dA equals the brute-force difference;
* a LIN1 path built by the exact trapezoid recurrence has A_d = 0;
* the gradient equals central finite differences of A, and vanishes at the
  closed-form posterior mean of a LIN1 window (the mode of a Gaussian).
"""

import numpy as np
import pytest

import workloads as W
from oracle import action as OA
from oracle import kalman as OK
from oracle.mp import action_mp


def _hh_state(M=12, seed=0, jitter=1.0):
    P = W.make_hh_problem(M, 0.02, 101, require_spike=False, init="truth")
    rng = np.random.default_rng(seed)
    X = P.X_true + jitter * rng.normal(size=P.X_true.shape) * np.array([0.5, 1e-3, 1e-3, 1e-3])
    X[:, 1:] = np.clip(X[:, 1:], 0.0, 1.0)
    p = P.p_true * (1.0 + 0.02 * rng.normal(size=7))
    return P, X, p


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_action_matches_mpmath(seed):
    P, X, p = _hh_state(M=10, seed=seed)
    spec = P.model.with_(beta=0.37)
    a = OA.action(spec, X, P.y, P.I, p)
    b = action_mp(spec, X, P.y, P.I, p)
    for u, v in zip(a, b):
        assert u == pytest.approx(v, rel=1e-13)
    assert a[0] == pytest.approx(a[1] + 0.37 * a[2], rel=1e-15)
    assert min(a) >= 0.0


def test_action_lin1_matches_mpmath():
    L = W.make_lin1_problem(M=9)
    a = OA.action(L.model, L.X_true, L.y, L.I, L.p0)
    b = action_mp(L.model, L.X_true, L.y, L.I, L.p0)
    for u, v in zip(a, b):
        assert u == pytest.approx(v, rel=1e-13)


def test_lin1_exact_recurrence_has_zero_model_error():
    L = W.make_lin1_problem(M=20)
    lam = L.p0[0]
    dt = L.model.dt
    a, b = 1 + lam * dt / 2, 1 - lam * dt / 2
    x = np.empty(21)
    x[0] = 0.7
    for n in range(1, 21):
        x[n] = (b * x[n - 1] + dt / 2 * (L.I[n] + L.I[n - 1])) / a
    A, A_o, A_d = OA.action(L.model, x[:, None], L.y, L.I, L.p0)
    assert A_d < 1e-26
    assert A_o > 0


@pytest.mark.parametrize("beta", [1.0, 0.05])
def test_local_delta_equals_bruteforce(beta):
    P, X, p = _hh_state(M=14, seed=5)
    spec = P.model.with_(beta=beta)
    M = P.M
    rng = np.random.default_rng(11)
    ns = np.arange(M + 1)
    xp = X + rng.normal(size=X.shape) * np.array([0.05, 5e-4, 5e-4, 5e-4])
    d = OA.delta_site(spec, X, P.y, P.I, p, ns, xp)
    A0 = OA.action(spec, X, P.y, P.I, p)[0]
    for n in ns:
        X2 = X.copy()
        X2[n] = xp[n]
        bf = OA.action(spec, X2, P.y, P.I, p)[0] - A0
        assert d[n] == pytest.approx(bf, rel=1e-9, abs=1e-9 * max(1.0, abs(A0)) * 1e-3), n


def test_local_delta_antisymmetric():
    P, X, p = _hh_state(M=8, seed=6)
    ns = np.arange(P.M + 1)
    xp = X + 0.01 * np.array([1.0, 1e-2, 1e-2, 1e-2])
    d1 = OA.delta_site(P.model, X, P.y, P.I, p, ns, xp)
    for n in ns:
        X2 = X.copy()
        X2[n] = xp[n]
        d2 = OA.delta_site(P.model, X2, P.y, P.I, p, [n], X[n:n + 1])[0]
        assert d1[n] == pytest.approx(-d2, rel=1e-12, abs=1e-12)


def test_param_delta_equals_bruteforce():
    P, X, p = _hh_state(M=30, seed=7)
    A0 = OA.action(P.model, X, P.y, P.I, p)[0]
    for l in range(7):
        pp = p.copy()
        pp[l] *= 1.001
        d = OA.delta_params(P.model, X, P.I, p, pp)
        bf = OA.action(P.model, X, P.y, P.I, pp)[0] - A0
        assert d == pytest.approx(bf, rel=1e-8, abs=1e-10 * A0), l


def test_gradient_matches_finite_differences():
    P, X, p = _hh_state(M=12, seed=8)
    spec = P.model.with_(beta=0.8)
    g, gp = OA.grad(spec, X, P.y, P.I, p)
    h = 1e-6
    scale = np.array([1.0, 1e-2, 1e-2, 1e-2])
    for n in range(P.M + 1):
        for c in range(4):
            X1 = X.copy()
            X2 = X.copy()
            X1[n, c] += h * scale[c]
            X2[n, c] -= h * scale[c]
            fd = (OA.action(spec, X1, P.y, P.I, p)[0] - OA.action(spec, X2, P.y, P.I, p)[0]) / (2 * h * scale[c])
            assert g[n, c] == pytest.approx(fd, rel=2e-5, abs=2e-5 * max(1.0, np.abs(g).max()) * 1e-2), (n, c)
    for l in range(7):
        dp = np.zeros(7)
        dp[l] = h * abs(p[l])
        fd = (OA.action(spec, X, P.y, P.I, p + dp)[0] - OA.action(spec, X, P.y, P.I, p - dp)[0]) / (2 * dp[l])
        assert gp[l] == pytest.approx(fd, rel=1e-5, abs=1e-6), l


def test_gradient_vanishes_at_lin1_posterior_mean():
    L = W.make_lin1_problem(M=24)
    mean, _ = OK.lin1_posterior(L.model, L.y, L.I, L.p0[0])
    g, _ = OA.grad(L.model, mean[:, None], L.y, L.I, L.p0)
    assert np.abs(g).max() < 1e-9
    g2, _ = OA.grad(L.model, mean[:, None] + 0.01, L.y, L.I, L.p0)
    assert np.abs(g2).max() > 1e-3
