"""Pins of the oracle sampler (Fig. 1, Sections 3.1 and 4.1-4.2).

* intra-colour order invariance (Section 4.1: same-parity sites may be
  updated in any order or simultaneously);
* exact detailed balance of each colour update and of the parameter move on
  a lattice-discretised window, with the acceptance probability taken from
  the oracle's own decision rule over the exact law of u; the composed sweep
  leaves the target invariant;
* whole sampler on the linear-Gaussian window: chain means and variances
  match the closed-form (Kalman-smoother) posterior within Monte Carlo error;
* HMC proposal: exact reversibility, O(e^2) energy error, and the same
  closed-form posterior;
* statistics and resumability (a split run equals one run bit for bit).
"""

import math

import numpy as np
import pytest

import workloads as W
from oracle import action as OA
from oracle import hmc as OH
from oracle import kalman as OK
from oracle import sampler as OS


def test_intra_colour_order_invariance():
    P = W.make_hh_problem(40, 0.02, 101, require_spike=False)
    X1 = P.X0.copy()
    p1 = P.p0.copy()
    X2 = P.X0.copy()
    p2 = P.p0.copy()
    kw = dict(seed=5, chain=2, sweep0=0, n_sweeps=6, w_state=P.w_state, w_param=P.w_param)
    OS.run(P.model, X1, p1, P.y, P.I, **kw)
    OS.run(P.model, X2, p2, P.y, P.I, order_rng=np.random.default_rng(0), **kw)
    np.testing.assert_allclose(X1, X2, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(p1, p2, rtol=1e-13)
    assert not np.array_equal(X1, P.X0)


def _accept_prob(dA):
    """P(accept) under the oracle's rule, for u = (c + 0.5) 2^-32 uniform over
    the 2^32 words c: count the words that accept (monotone in c)."""
    if not np.isfinite(dA):
        return 0.0
    lo, hi = 0, 1 << 32          # accepts(c) true for c < cut
    while lo < hi:
        mid = (lo + hi) // 2
        u = (mid + 0.5) * 2.0 ** -32
        if OS.accepts(np.float64(u), dA):
            lo = mid + 1
        else:
            hi = mid
    return lo / 2.0 ** 32


def test_detailed_balance_on_lattice():
    """LIN1, M=1 (sites 0 and 1) plus its parameter, K=7 levels each."""
    K = 7
    L = W.make_lin1_problem(M=1, Rd=3.0, Ro=2.0)
    spec = L.model.with_(p_mask=1, p_lo=(0.3,), p_hi=(0.9,))
    x_lv = np.linspace(-1.0, 1.0, K)
    p_lv = np.linspace(0.3, 0.9, K)
    states = [(i, j, k) for i in range(K) for j in range(K) for k in range(K)]
    index = {s: t for t, s in enumerate(states)}
    S = len(states)

    def X_of(s):
        return np.array([[x_lv[s[0]]], [x_lv[s[1]]]]), np.array([p_lv[s[2]]])

    A = np.array([OA.action(spec, *X_of(s)[:1], L.y, L.I, X_of(s)[1])[0] for s in states])
    pi = np.exp(-(A - A.min()))
    pi /= pi.sum()

    def kernel(coord):
        T = np.zeros((S, S))
        for s in states:
            a = index[s]
            X, p = X_of(s)
            for step in (-1, 1):
                t = list(s)
                t[coord] += step
                if not 0 <= t[coord] < K:
                    T[a, a] += 0.5      # leaves the box: rejected
                    continue
                X2, p2 = X_of(tuple(t))
                if coord < 2:
                    dA = OA.delta_site(spec, X, L.y, L.I, p, [coord], X2[coord:coord + 1])[0]
                else:
                    dA = OA.delta_params(spec, X, L.I, p, p2)
                q = _accept_prob(dA)
                T[a, index[tuple(t)]] += 0.5 * q
                T[a, a] += 0.5 * (1 - q)
        return T

    Ts = [kernel(c) for c in range(3)]
    for T in Ts:
        np.testing.assert_allclose(T.sum(axis=1), 1.0, atol=1e-15)
        F = pi[:, None] * T
        np.testing.assert_allclose(F, F.T, atol=1e-9 * pi.max())
    sweep = Ts[0] @ Ts[1] @ Ts[2]
    np.testing.assert_allclose(pi @ sweep, pi, atol=1e-9 * pi.max())
    # the composed sweep is invariant but not reversible in general
    Fs = pi[:, None] * sweep
    assert np.abs(Fs - Fs.T).max() > 1e-6 * pi.max()


def _batch_mcse(trace, nb=40):
    n = trace.shape[0] // nb * nb
    b = trace[:n].reshape(nb, -1, *trace.shape[1:]).mean(axis=1)
    return b.std(axis=0, ddof=1) / np.sqrt(nb)


@pytest.mark.slow
def test_lin1_sampler_matches_closed_form():
    L = W.make_lin1_problem(M=16, w=0.25)
    mean, var = OK.lin1_posterior(L.model, L.y, L.I, L.p0[0])
    X = L.X0.copy()
    p = L.p0.copy()
    kw = dict(seed=L.seed, chain=0, w_state=L.w_state, w_param=L.w_param, flags=OS.STATES)
    OS.run(L.model, X, p, L.y, L.I, sweep0=0, n_sweeps=500, **kw)
    n = 16000
    tr = np.empty((n, 17))
    for i in range(n):
        OS.run(L.model, X, p, L.y, L.I, sweep0=500 + i, n_sweeps=1, **kw)
        tr[i] = X[:, 0]
    m = tr.mean(axis=0)
    se = _batch_mcse(tr)
    z = (m - mean) / se
    assert np.abs(z).max() < 4.5, z
    v = tr.var(axis=0)
    se_v = _batch_mcse((tr - m) ** 2)
    zv = (v - var) / se_v
    assert np.abs(zv).max() < 4.5, zv


def test_hmc_leapfrog_reversible_and_second_order():
    P = W.make_hh_problem(24, 0.02, 101, require_spike=False, init="truth")
    spec = P.model
    minv_s = np.array([0.05, 1e-6, 1e-6, 1e-6]) ** 2 * 1e2
    minv_p = (1e-3 * np.abs(P.p_true)) ** 2
    r, rp, mask = OH.momenta(spec, 3, 0, 0, P.M, minv_s, minv_p)
    e = 0.02
    q, qp, r1, rp1, _ = OH.leapfrog(spec, P.X_true, P.p_true, P.y, P.I, r, rp, mask, e, 10, minv_s, minv_p)
    q2, qp2, r2, rp2, _ = OH.leapfrog(spec, q, qp, P.y, P.I, -r1, -rp1, mask, e, 10, minv_s, minv_p)
    np.testing.assert_allclose(q2, P.X_true, rtol=0, atol=1e-10 * np.abs(P.X_true).max())
    np.testing.assert_allclose(qp2, P.p_true, rtol=1e-10)
    np.testing.assert_allclose(-r2, r, rtol=1e-7, atol=1e-7 * np.abs(r).max())

    def dH(eps, L):
        H0 = OA.action(spec, P.X_true, P.y, P.I, P.p_true)[0] + OH.kinetic(r, rp, minv_s, minv_p)
        q, qp, r1, rp1, _ = OH.leapfrog(spec, P.X_true, P.p_true, P.y, P.I, r, rp, mask, eps, L, minv_s, minv_p)
        return OA.action(spec, q, P.y, P.I, qp)[0] + OH.kinetic(r1, rp1, minv_s, minv_p) - H0

    d1 = abs(dH(0.004, 10))
    d2 = abs(dH(0.002, 20))
    assert 2.5 < d1 / d2 < 6.0, (d1, d2)


def test_hmc_reflection_reversible():
    """Trajectories that cross the gate walls (m comes within 1e-3 of 1 at
    the spike peak) are reflected, stay valid, and run back exactly under
    r -> -r."""
    P = W.make_hh_problem(400, 0.02, 101, init="truth")
    spec = P.model
    assert 1.0 - P.X_true[:, 1].max() < 1e-3
    minv_s = np.array([2.5e-3, 1e-4, 1e-4, 1e-4])
    minv_p = (1e-3 * np.abs(P.p_true)) ** 2
    r, rp, mask = OH.momenta(spec, 5, 0, 0, P.M, minv_s, minv_p)
    cnt = [0]
    q, qp, r1, rp1, ok = OH.leapfrog(spec, P.X_true, P.p_true, P.y, P.I, r, rp, mask, 0.02, 10, minv_s, minv_p,
                                     count=cnt)
    assert ok and cnt[0] > 0
    assert (q[:, 1:] >= 0).all() and (q[:, 1:] <= 1).all()
    cnt2 = [0]
    q2, qp2, r2, rp2, ok2 = OH.leapfrog(spec, q, qp, P.y, P.I, -r1, -rp1, mask, 0.02, 10, minv_s, minv_p,
                                        count=cnt2)
    assert ok2 and cnt2[0] == cnt[0]
    np.testing.assert_allclose(q2, P.X_true, rtol=0, atol=1e-10 * np.abs(P.X_true).max())
    np.testing.assert_allclose(qp2, P.p_true, rtol=1e-10)
    np.testing.assert_allclose(-r2, r, rtol=1e-7, atol=1e-7 * np.abs(r).max())


def test_hmc_reflection_samples_truncated_posterior():
    """HMC with reflecting walls samples the box-truncated posterior: LIN1
    with M = 1 (two coordinates), moments against a fine grid integral of
    exp(-A) over the box, A written from the LIN1 definition."""
    L = W.make_lin1_problem(M=1, dt=0.1, Rd=100.0, Ro=4.0, data_seed=3)
    lam, dt, Rd, Ro = L.p0[0], L.model.dt, L.model.Rd[0], L.model.Ro
    a, b = 1 + lam * dt / 2, 1 - lam * dt / 2
    k1 = 0.5 * dt * (L.I[1] + L.I[0])
    y1 = L.y[1]
    lo, hi = y1 - 0.35, y1 + 0.25
    spec = L.model.with_(x_lo=(lo,), x_hi=(hi,))
    g = np.linspace(lo, hi, 1601)
    x0, x1 = np.meshgrid(g, g, indexing="ij")
    A = 0.5 * Ro * (y1 - x1) ** 2 + 0.5 * Rd * (a * x1 - b * x0 - k1) ** 2
    wgt = np.exp(-(A - A.min()))
    wgt[0, :] *= 0.5
    wgt[-1, :] *= 0.5
    wgt[:, 0] *= 0.5
    wgt[:, -1] *= 0.5
    Z = wgt.sum()
    m_ref = np.array([(wgt * x0).sum(), (wgt * x1).sum()]) / Z
    v_ref = np.array([(wgt * (x0 - m_ref[0]) ** 2).sum(), (wgt * (x1 - m_ref[1]) ** 2).sum()]) / Z
    X = np.array([[y1], [y1]])
    p = L.p0.copy()
    n = 6000
    tr = np.empty((n, 2))
    acc = 0
    cnt = 0
    for k in range(n):
        if k < 500:
            r, rp, mask = OH.momenta(spec, 12, 0, k, 1, [0.04], [1.0])
            c = [0]
            OH.leapfrog(spec, X, p, L.y, L.I, r, rp, mask, 0.12, 6, [0.04], [1.0], count=c)
            cnt += c[0]
        X, p, okp, _ = OH.hmc_proposal(spec, X, p, L.y, L.I, seed=12, chain=0, k=k, e=0.12, L=6,
                                       minv_state=[0.04], minv_param=[1.0])
        acc += okp
        tr[k] = X[:, 0]
    assert cnt > 25               # the walls are hit often
    assert acc / n > 0.5
    m = tr.mean(axis=0)
    z = (m - m_ref) / _batch_mcse(tr, 30)
    assert np.abs(z).max() < 4.5, (m, m_ref, z)
    zv = (tr.var(axis=0) - v_ref) / _batch_mcse((tr - m) ** 2, 30)
    assert np.abs(zv).max() < 4.5, zv


@pytest.mark.slow
def test_hmc_lin1_matches_closed_form():
    L = W.make_lin1_problem(M=16)
    mean, var = OK.lin1_posterior(L.model, L.y, L.I, L.p0[0])
    X = mean[:, None].copy()
    p = L.p0.copy()
    minv = np.array([float(np.median(var))])
    n = 3000
    tr = np.empty((n, 17))
    acc = 0
    for k in range(n):
        X, p, ok, _ = OH.hmc_proposal(L.model, X, p, L.y, L.I, seed=9, chain=0, k=k,
                                      e=0.35, L=8, minv_state=minv, minv_param=np.array([1.0]))
        acc += ok
        tr[k] = X[:, 0]
    assert 0.5 < acc / n < 1.0
    m = tr.mean(axis=0)
    z = (m - mean) / _batch_mcse(tr, 30)
    assert np.abs(z).max() < 4.5, z
    zv = (tr.var(axis=0) - var) / _batch_mcse((tr - m) ** 2, 30)
    assert np.abs(zv).max() < 4.5, zv


def test_stats_and_resume_bitwise():
    P = W.make_hh_problem(20, 0.02, 101, require_spike=False)
    kw = dict(seed=11, chain=4, w_state=P.w_state, w_param=P.w_param)
    Xa, pa = P.X0.copy(), P.p0.copy()
    st = OS.Stats(P.M, 4, 7, 10, burn=4, xref=P.X0.copy())
    OS.run(P.model, Xa, pa, P.y, P.I, sweep0=0, n_sweeps=10, stats=st, **kw)
    Xb, pb = P.X0.copy(), P.p0.copy()
    s1 = OS.Stats(P.M, 4, 7, 6, burn=4, xref=P.X0.copy())
    OS.run(P.model, Xb, pb, P.y, P.I, sweep0=0, n_sweeps=6, stats=s1, **kw)
    s2 = OS.Stats(P.M, 4, 7, 4, burn=4, xref=P.X0.copy())
    OS.run(P.model, Xb, pb, P.y, P.I, sweep0=6, n_sweeps=4, stats=s2, **kw)
    assert np.array_equal(Xa, Xb) and np.array_equal(pa, pb)
    np.testing.assert_array_equal(st.ptrace, np.concatenate([s1.ptrace, s2.ptrace]))
    np.testing.assert_allclose(st.sum, s1.sum + s2.sum, rtol=1e-15, atol=1e-300)
    assert st.n_post == 6
    assert st.acc[:2].sum() > 0
    # moments equal the direct computation from recorded paths
    Xc, pc = P.X0.copy(), P.p0.copy()
    S = np.zeros_like(Xc)
    Q = np.zeros_like(Xc)
    for k in range(10):
        OS.run(P.model, Xc, pc, P.y, P.I, sweep0=k, n_sweeps=1, **kw)
        if k >= 4:
            S += Xc - P.X0
            Q += (Xc - P.X0) ** 2
    np.testing.assert_allclose(st.sum, S, rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(st.sumsq, Q, rtol=1e-14, atol=1e-20)


def test_batch_sums_from_recorded_paths():
    # sweeps k = 2 .. 14, burn 3, stride 2: samples after sweeps 3, 5, 7, 9,
    # 11, 13 (six), split into four runs of consecutive samples of sizes
    # 2, 1, 2, 1 (sample i in batch i * 4 // 6)
    P = W.make_hh_problem(12, 0.02, 101, require_spike=False)
    kw = dict(seed=5, chain=2, w_state=P.w_state, w_param=P.w_param)
    X, p = P.X0.copy(), P.p0.copy()
    st = OS.Stats(P.M, 4, 7, 13, burn=3, stride=2, nbatch=4, xref=P.X0.copy())
    OS.run(P.model, X, p, P.y, P.I, sweep0=2, n_sweeps=13, stats=st, **kw)
    Xc, pc = P.X0.copy(), P.p0.copy()
    want = np.zeros((4,) + Xc.shape)
    which = {3: 0, 5: 0, 7: 1, 9: 2, 11: 2, 13: 3}
    for k in range(2, 15):
        OS.run(P.model, Xc, pc, P.y, P.I, sweep0=k, n_sweeps=1, **kw)
        if k in which:
            want[which[k]] += Xc - P.X0
    assert st.n_post == 6
    np.testing.assert_allclose(st.batch, want, rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(st.batch.sum(axis=0), st.sum, rtol=1e-13, atol=1e-13)


def test_out_of_box_proposals_are_rejected():
    P = W.make_hh_problem(16, 0.02, 101, require_spike=False)
    spec = P.model.with_(x_lo=(-100.0, 0.0, 0.0, 0.0), x_hi=(200.0, 1e-9, 1.0, 1.0))
    X = P.X0.copy()
    X[:, 1] = 0.0
    dbg = OS.Debug()
    OS.run(spec, X, P.p0.copy(), P.y, P.I, seed=1, chain=0, sweep0=0, n_sweeps=1,
           w_state=P.w_state, w_param=P.w_param, debug=dbg)
    out = (dbg.xprop[:, 1] < 0) | (dbg.xprop[:, 1] > 1e-9)
    assert out.any()
    assert not dbg.accept[out].any()
    assert np.isnan(dbg.dA[out]).all()
