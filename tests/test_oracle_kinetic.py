"""Pins of the Table 1 kinetic-constant moves (oracle/sampler.kinetic_moves).

* The change of the action under a move of one constant equals the 50-digit
  mpmath action difference (oracle/mp.py evaluates the gate equations of
  Section 5.1 from the definitions, with its own tanh).
* Only the changed gate's model error moves: a move of an m constant leaves
  the h and n terms alone.
* The Metropolis chain of one constant, with the path and every other
  constant held fixed, samples exp(-A) over its box: its mean and variance
  match a quadrature of exp(-A) on a grid (a wrong sign of dA, an asymmetric
  proposal or a dropped term shifts them).
"""

import numpy as np
import pytest

import workloads as W
from oracle import action as OA
from oracle import mp as OMP
from oracle import sampler as OS


def _window(M, seed=101):
    return W.make_hh_problem(M, 0.02, seed, require_spike=False, init="truth")


@pytest.mark.parametrize("i", [0, 1, 2, 3, 5, 8, 11])
def test_delta_kinetic_equals_mpmath(i):
    prob = _window(6)
    spec = prob.model
    X = prob.X_true + 0.01
    X[:, 1:] = np.clip(X[:, 1:], 0, 1)
    kin = np.array(spec.gates, dtype=np.float64).ravel()
    new = kin.copy()
    new[i] *= 1.07
    d = OA.delta_kinetic(spec, X, prob.I, prob.p_true, new.reshape(3, 4))
    a0 = OMP.action_mp(spec, X, prob.y, prob.I, prob.p_true)
    a1 = OMP.action_mp(spec.with_(gates=tuple(tuple(g) for g in new.reshape(3, 4))), X, prob.y, prob.I,
                       prob.p_true)
    ref = float(a1[0] - a0[0]) if isinstance(a0, (tuple, list)) else float(a1 - a0)
    assert d == pytest.approx(ref, rel=1e-9, abs=1e-12)


def test_kinetic_move_touches_only_its_gate():
    prob = _window(30)
    spec = prob.model
    kin = np.array(spec.gates, dtype=np.float64).ravel()
    new = kin.copy()
    new[4] += 0.3                        # V_a of h
    mod0 = OA.model_for(spec)
    mod1 = OA.model_for(spec.with_(gates=tuple(tuple(g) for g in new.reshape(3, 4))))
    F0 = mod0.F(prob.X_true, prob.I, prob.p_true)
    F1 = mod1.F(prob.X_true, prob.I, prob.p_true)
    np.testing.assert_array_equal(F0[:, [0, 1, 3]], F1[:, [0, 1, 3]])
    assert np.abs(F0[:, 2] - F1[:, 2]).max() > 0


@pytest.mark.slow
@pytest.mark.parametrize("i", [0, 9])
def test_kinetic_chain_samples_the_conditional(i):
    prob = _window(20, seed=103)
    lo = list(prob.model.k_lo)
    hi = list(prob.model.k_hi)
    kin0 = np.array(prob.model.gates, dtype=np.float64).ravel()
    spec = prob.model.with_(k_mask=1 << i, Rd=(100.0, 1e3, 1e3, 1e3))
    X = prob.X_true
    # quadrature of exp(-A) over the constant's box
    v = np.linspace(lo[i], hi[i], 4001)
    dA = np.empty(len(v))
    for j, vj in enumerate(v):
        g = kin0.copy()
        g[i] = vj
        dA[j] = OA.delta_kinetic(spec, X, prob.I, prob.p_true, g.reshape(3, 4))
    wq = np.exp(-(dA - dA.min()))
    m_q = (wq * v).sum() / wq.sum()
    v_q = (wq * (v - m_q) ** 2).sum() / wq.sum()
    # the Metropolis chain of that constant alone
    kin = kin0.copy()
    kin[i] = m_q
    w_kin = np.full(12, 2.0 * np.sqrt(v_q))
    p = np.asarray(prob.p_true, dtype=np.float64).copy()
    Xc = X.copy()
    n = 6000
    tr = np.empty(n)
    for k in range(n):
        OS.run(spec, Xc, p, prob.y, prob.I, seed=5, chain=0, sweep0=k, n_sweeps=1, w_state=prob.w_state,
               w_param=prob.w_param, flags=OS.KINETIC, kin=kin, w_kin=w_kin)
        tr[k] = kin[i]
    np.testing.assert_array_equal(Xc, X)
    b = tr[1000:].reshape(50, -1).mean(axis=1)
    se = b.std(ddof=1) / np.sqrt(len(b))
    assert abs(tr[1000:].mean() - m_q) < 4.0 * se + 1e-12
    assert abs(tr[1000:].var() / v_q - 1.0) < 0.15
