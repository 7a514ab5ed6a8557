"""The FP32 HMC trajectory, element by element, at the 64-chain M = 16384 shape.

One proposal of 20 leapfrog steps for 64 chains (the HMC workload's launch
shape), with every intermediate state recorded by the library.  Each step is
checked against the oracle's leapfrog arithmetic applied to the GPU's own
state before that step (as the FP32 site updates are checked on the GPU's own
proposals): the drift and its reflection at the box walls, the kick with the
action gradient evaluated by the oracle in FP64, and the parameter drift and
kick with the chain-summed dA/dp.  The bar for every coordinate is the
rounding of one FP32 step: a few u = 2^-24 of every magnitude formed, plus
the step size times the first-order FP32 bound of the gradient
(tests/fp32_bounds.py).  Coordinates whose drift ends within rounding of a
box wall (where the reflection decision is a tie) are counted and excluded.
Momenta drawn at the start use FP32 Box-Muller and get its error bound
(largest where u_a is close to 1, where the square root amplifies the
rounding of the logarithm).
"""

import numpy as np
import pytest

import workloads as W
from oracle import action as OA
from oracle import hmc as OH
from oracle import philox as ph

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1103_4887_amd")

pytestmark = pytest.mark.gpu

U = 2.0 ** -24


@pytest.fixture(scope="module")
def ctx():
    c = P.Context(0)
    yield c
    c.close()


def test_hmc_fp32_trajectory_elementwise_c5_shape(ctx):
    import fp32_bounds as FB

    prob = W.config_problem("c5", init="truth")
    spec = prob.model
    B, L = 64, 20
    M = prob.M
    rng = np.random.default_rng(5)
    # mid-run states: the truth perturbed on the posterior's scale, per chain
    starts = []
    for _ in range(B):
        X = prob.X_true + rng.normal(size=prob.X_true.shape) * np.array([0.2, 1e-3, 1e-3, 1e-3])
        X[:, 1:] = np.clip(X[:, 1:], 1e-4, 1.0 - 1e-4)   # inside the box, off its walls
        starts.append(X.astype(np.float32).astype(np.float64))
    p0 = np.asarray(prob.p_true) * (1.0 + 0.005 * rng.standard_normal(7))
    minv = np.array([0.3, 1e-5, 1e-5, 1e-5] + list((1e-3 * np.abs(np.asarray(W.P_STAR))) ** 2))
    eps, seed, k0 = 0.02, 909, 3
    chains = list(range(100, 100 + B))
    batch = P.PackedBatch.pack(starts, [p0] * B, [prob.y] * B, [prob.I] * B, chains, "fp32")
    st = P.HmcStats.allocate(B, 1, trajectory=batch, L_steps=L)
    print(f"hmc fp32 trajectory: {B} chains x M={M}, L={L}", flush=True)
    P.pimc_hmc(ctx, spec, batch, seed=seed, k0=k0, eps=eps, L_steps=L, minv=minv, n_proposals=1, stats=st)
    assert ctx.sync() == 0
    S1 = M + 1
    tq = st.traj_q.cpu().numpy().astype(np.float64).reshape(L + 1, B, S1, 4)
    tr = st.traj_r.cpu().numpy().astype(np.float64).reshape(L + 1, B, S1, 4)
    tp = st.traj_p.cpu().numpy()
    trp = st.traj_rp.cpu().numpy()
    acc = st.acc.cpu().numpy()
    Xend = batch.X.cpu().numpy().astype(np.float64).reshape(B, S1, 4)
    pend = batch.p.cpu().numpy()
    assert np.isfinite(tq).all() and np.isfinite(tr).all()
    y32 = prob.y.astype(np.float32).astype(np.float64)
    I32 = prob.I.astype(np.float32).astype(np.float64)
    lo, hi = np.asarray(spec.x_lo)[None, :], np.asarray(spec.x_hi)[None, :]
    plo, phi = np.asarray(spec.p_lo), np.asarray(spec.p_hi)
    ms, mp_ = minv[:4][None, :], minv[4:]
    mask = np.array([(spec.p_mask >> l) & 1 for l in range(7)], dtype=bool)

    def grad_and_bound(q, p):
        g, gp = OA.grad(spec, q, y32, I32, p)
        gb, gpb = FB.grad_bound(spec, q, y32, I32, p)
        # dA/dp: per-site FP32 products summed in FP64
        return g, gp, gb, gpb + 16 * U * np.abs(gp)

    def p_flip(s, b):
        """rp(s-1/2) after the reflection of drift s (s >= 1), from the GPU's p(s-1)."""
        pre = tp[s - 1, b] + eps * mp_ * trp[s, b]
        out = trp[s, b].copy()
        _, fl, _, _ = OH.reflect(pre[mask], out[mask], plo[mask], phi[mask])
        out[mask] = fl
        return out

    worst = {"q": 0.0, "r": 0.0, "rp": 0.0}
    ties = 0
    full = set(range(0, B, 8))    # every step for eight chains, steps 1, 2, L for all
    for b in range(B):
        np.testing.assert_array_equal(tq[0, b], starts[b])
        np.testing.assert_array_equal(tp[0, b], p0)
        r0, rp0, _ = OH.momenta(spec, seed, chains[b], k0, M, minv[:4], minv[4:])
        # FP64 Box-Muller on both sides (a few ulp of the library functions)
        np.testing.assert_allclose(trp[0, b], rp0, rtol=1e-12, atol=1e-12 * np.abs(rp0).max())
        # r(1/2) = r0 - e/2 g(q0), r0 from FP32 Box-Muller (4e-6 of |z| and absolute)
        g0, _, gb0, _ = grad_and_bound(starts[b], p0)
        zb = FB.box_muller_bound(ph.draw(seed, chains[b], np.arange(M + 1), k0, ph.TAG_MOM))
        ref = r0 - 0.5 * eps * g0
        tol = zb / np.sqrt(minv[:4])[None, :] + 0.5 * eps * gb0 + 4 * U * (
            np.abs(ref) + np.abs(r0) + 0.5 * eps * np.abs(g0))
        err = np.abs(tr[0, b] - ref)
        worst["r"] = max(worst["r"], float((err / tol).max()))
        assert (err <= tol).all(), ("r(1/2)", b, np.unravel_index(np.argmax(err / tol), err.shape))
        for s in (range(1, L + 1) if b in full else (1, 2, L)):
            q_prev, r_prev = tq[s - 1, b], tr[s - 1, b]
            # drift and reflection of the positions
            step = eps * ms * r_prev
            pre = q_prev + step
            q_ref, r_flip, _, _ = OH.reflect(pre, r_prev, lo, hi)
            tolq = 4 * U * (np.abs(q_prev) + np.abs(step) + np.abs(pre) + np.abs(q_ref))
            tie = (np.abs(pre - lo) <= 2 * tolq) | (np.abs(pre - hi) <= 2 * tolq)
            ok = ~tie
            ties += int(tie.sum())
            err = np.abs(tq[s, b] - q_ref)
            worst["q"] = max(worst["q"], float((err[ok] / tolq[ok]).max()))
            assert (err[ok] <= tolq[ok]).all(), ("q", s, b, np.unravel_index(np.argmax(err / tolq), err.shape))
            # parameters: FP64 drift from the GPU's p(s-1), rp(s-1/2)
            p_pre = tp[s - 1, b] + eps * mp_ * trp[s, b]
            p_ref, _, _, _ = OH.reflect(p_pre[mask], trp[s, b][mask], plo[mask], phi[mask])
            np.testing.assert_allclose(tp[s, b][mask], p_ref, rtol=1e-13, atol=0)
            # parameter kick that formed rp(s-1/2), with dA/dp at the GPU's q(s-1), p(s-1)
            rp_before = trp[0, b] if s == 1 else p_flip(s - 1, b)
            c = 0.5 if s == 1 else 1.0
            _, gp_prev, _, gpb_prev = grad_and_bound(q_prev, tp[s - 1, b])
            rp_ref = rp_before - c * eps * gp_prev
            tolp = c * eps * gpb_prev + 1e-13 * np.abs(rp_ref)
            errp = np.abs(trp[s, b] - rp_ref)
            worst["rp"] = max(worst["rp"], float((errp[mask] / tolp[mask]).max()))
            assert (errp[mask] <= tolp[mask]).all(), ("rp", s, b, errp, tolp)
            # kick of the site momenta with the gradient at the GPU's q(s), p(s)
            g, gp, gb, gpb = grad_and_bound(tq[s, b], tp[s, b])
            kick = eps if s < L else 0.5 * eps
            ref = r_flip - kick * g
            tol = kick * gb + 4 * U * (np.abs(ref) + np.abs(r_flip) + kick * np.abs(g))
            err = np.abs(tr[s, b] - ref)
            worst["r"] = max(worst["r"], float((err[ok] / tol[ok]).max()))
            assert (err[ok] <= tol[ok]).all(), ("r", s, b, np.unravel_index(np.argmax(err / tol), err.shape))
            if s == L:
                rp_end = p_flip(L, b) - 0.5 * eps * gp
                tole = 0.5 * eps * gpb + 1e-13 * np.abs(rp_end)
                erre = np.abs(trp[L + 1, b] - rp_end)
                worst["rp"] = max(worst["rp"], float((erre[mask] / tole[mask]).max()))
                assert (erre[mask] <= tole[mask]).all(), ("rp(L)", b, erre, tole)
        # the proposal's outcome is the end of the trajectory or its start, exactly
        src = L if acc[b, 0] else 0
        np.testing.assert_array_equal(Xend[b], tq[src, b])
        np.testing.assert_array_equal(pend[b], tp[src, b])
    print(f"hmc fp32 trajectory: worst error / bound {worst}, wall ties excluded {ties}, "
          f"accepted {int(acc[:, 0].sum())} of {B}", flush=True)
    # the true m comes within about 2e-4 of 1 at every spike, so a few drifts
    # end within rounding of that wall
    checked = B * (M + 1) * 4 * 3 + 8 * (M + 1) * 4 * (L - 3)
    assert ties <= 1e-4 * checked, ties
