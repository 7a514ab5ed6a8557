"""Pins of the model checks (oracle/diagnostics.py).

* The model errors of the true path of a window built by the trapezoid
  recurrence of the linear-Gaussian model are the noise that built it
  (exactly, up to rounding); the observation errors are y - V.
* Heun's method has global error O(dt^2): halving dt quarters the distance
  to a fine RK4 reference; with zero noise the ensemble collapses onto the
  deterministic forecast, and with noise its one-step spread is 1/sqrt(Rd).
"""

import numpy as np

import workloads as W
from oracle import diagnostics as OD
from oracle import philox as ph


def test_model_errors_of_a_trapezoid_path_are_its_noise():
    L = W.make_lin1_problem(M=30)
    lam = L.meta["lam"]
    dt = L.model.dt
    rng = np.random.default_rng(3)
    e_true = rng.standard_normal(30) * 0.1
    x = np.empty(31)
    x[0] = 0.7
    a, b = 1 + lam * dt / 2, 1 - lam * dt / 2
    for n in range(1, 31):
        k = 0.5 * dt * (L.I[n] + L.I[n - 1])
        x[n] = (b * x[n - 1] + k + e_true[n - 1]) / a
    e, d = OD.model_errors(L.model, x[:, None], L.y, L.I, np.array([lam]))
    np.testing.assert_allclose(e[:, 0], e_true, rtol=0, atol=1e-13)
    np.testing.assert_allclose(d, L.y[1:] - x[1:], rtol=0, atol=0)


def test_heun_forecast_second_order_and_noise():
    prob = W.make_hh_problem(64, 0.02, 101, require_spike=False, init="truth")
    spec = prob.model
    x0 = prob.X_true[10]
    T = 4.0                                   # ms
    errs = []
    for dt in (0.02, 0.01, 0.005):
        n = int(round(T / dt))
        I = np.full(n + 1, 8.0)
        fc = OD.forecast(spec.with_(dt=dt), x0, prob.p_true, I, n)
        ref = OD.forecast(spec.with_(dt=dt / 16), x0, prob.p_true, np.full(16 * n + 1, 8.0), 16 * n)[-1]
        errs.append(np.abs(fc[-1] - ref).max())
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0, errs
    I = np.full(11, 8.0)
    det = OD.forecast(spec, x0, prob.p_true, I, 10)
    one = OD.forecast(spec, x0, prob.p_true, I, 10, noise=0.0, seed=5, member=3)
    np.testing.assert_array_equal(det, one)
    # one noisy step: the deviation from the deterministic step is the
    # Philox normals scaled by 1/sqrt(Rd)
    st = OD.forecast(spec, x0, prob.p_true, I, 1, noise=1.0, seed=5, member=3)
    z = ph.normals4(ph.draw(5, 0, 3, 0, OD.TAG_FCST))[0]
    np.testing.assert_allclose(st[1] - det[1], z / np.sqrt(np.asarray(spec.Rd)), rtol=1e-12, atol=1e-15)
