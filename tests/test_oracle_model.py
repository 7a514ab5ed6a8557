"""Pins of the oracle's HH vector field, Jacobian and dF/dp (Section 5.1).

* special values of the gating functions fixed by their definitions:
  a_inf(V_a) = 1/2, tau_a(V_a) = tau0 + tau1, F_a = 0 at a = a_inf(V);
* dV/dt special cases: with all gates closed the Na and K currents vanish,
  at V = p7 the leak vanishes, and so on;
* J and dF/dp agree with central finite differences of F;
* the trapezoid model error of the RK4 truth path (a separate integrator of
  the same equations in `workloads`) is O(dt^3): small away from spikes and
  shrinking eightfold when dt halves.
"""

import numpy as np
import pytest

import workloads as W
from oracle.action import eps
from oracle.models import HH

P = np.array(W.P_STAR)
G = W.GATES_MHN


def test_gate_special_values():
    hh = HH(G)
    for j, (Va, dVa, t0, t1) in enumerate(G):
        X = np.array([[Va, 0.2, 0.3, 0.4]])
        _, ainf, tau = hh._gate(X[:, 0], j)
        assert ainf[0] == 0.5
        assert tau[0] == t0 + t1
        # far from V_a the gate saturates at 0 or 1 with tau -> tau0
        far = hh._gate(np.array([Va + 40 * abs(dVa)]), j)
        assert far[2][0] == pytest.approx(t0, rel=1e-12)
        assert far[1][0] == pytest.approx(1.0 if dVa > 0 else 0.0, abs=1e-12)


def test_gate_fixed_point():
    hh = HH(G)
    V = np.linspace(-20, 110, 27)
    X = np.zeros((len(V), 4))
    X[:, 0] = V
    for j in range(3):
        X[:, 1 + j] = hh._gate(V, j)[1]
    F = hh.F(X, np.zeros(len(V)), P)
    assert np.abs(F[:, 1:]).max() < 1e-15


def test_voltage_equation_special_cases():
    hh = HH(G)
    I = np.array([3.5])
    # gates closed: only drive and leak remain
    X = np.array([[7.0, 0.0, 0.9, 0.0]])
    assert hh.F(X, I, P)[0, 0] == pytest.approx(P[0] * 3.5 + P[5] * (P[6] - 7.0), rel=1e-15)
    # at V = p7 with closed gates only the drive remains
    X = np.array([[P[6], 0.0, 0.5, 0.0]])
    assert hh.F(X, I, P)[0, 0] == pytest.approx(P[0] * 3.5, rel=1e-15)
    # fully open m, h, n at V = p3: the Na current vanishes
    X = np.array([[P[2], 1.0, 1.0, 1.0]])
    expect = P[3] * (P[4] - P[2]) + P[5] * (P[6] - P[2])
    assert hh.F(X, np.zeros(1), P)[0, 0] == pytest.approx(expect, rel=1e-14)
    # F is affine in p1 with slope I
    Pp = P.copy()
    Pp[0] += 1.0
    X = np.array([[20.0, 0.3, 0.4, 0.5]])
    assert hh.F(X, I, Pp)[0, 0] - hh.F(X, I, P)[0, 0] == pytest.approx(3.5, rel=1e-12)


def test_jacobian_and_dFdp_by_finite_differences():
    hh = HH(G)
    rng = np.random.default_rng(3)
    N = 40
    X = np.column_stack([rng.uniform(-20, 110, N), rng.uniform(0, 1, (N, 3))])
    I = rng.normal(5, 3, N)
    J = hh.J(X, P)
    h = 1e-6
    for b in range(4):
        dx = np.zeros(4)
        dx[b] = h * (10.0 if b == 0 else 0.01)
        fd = (hh.F(X + dx, I, P) - hh.F(X - dx, I, P)) / (2 * dx[b])
        np.testing.assert_allclose(J[:, :, b], fd, rtol=1e-6, atol=1e-6)
    dFp = hh.dF_dp(X, I, P)
    for l in range(7):
        dp = np.zeros(7)
        dp[l] = 1e-6 * abs(P[l])
        fd = (hh.F(X, I, P + dp) - hh.F(X, I, P - dp)) / (2 * dp[l])
        np.testing.assert_allclose(dFp[:, :, l], fd, rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("dt", [0.02, 0.01])
def test_truth_path_satisfies_trapezoid_rule(dt):
    """eps_n of the RK4 truth is the trapezoid local error, O(dt^3)."""
    M = int(round(6.0 / dt))
    prob = W.make_hh_problem(M, dt, 101, require_spike=False, init="truth")
    e = eps(HH(G), prob.X_true, prob.I, P, dt)
    scale = np.abs(prob.X_true[1:] - prob.X_true[:-1]).max(axis=0)
    assert (np.abs(e).max(axis=0) < 0.05 * scale).all()
    if dt == 0.01:
        prob2 = W.make_hh_problem(M // 2, 0.02, 101, require_spike=False, init="truth")
        e2 = eps(HH(G), prob2.X_true, prob2.I, P, 0.02)
        # the stimulus differs (new OU draws), so compare the bulk size only
        r = np.median(np.abs(e2[:, 0])) / np.median(np.abs(e[:, 0]))
        assert 3.0 < r < 20.0
