"""HMC proposals of the HIP library against the oracle's leapfrog/HMC.

FP64: the decision of every chain equals the oracle's wherever
|dH + log u| > 1e-6, dH agrees to 1e-8 relative (plus 1e-9 absolute), final
positions and parameters to 1e-10.  FP32 trajectories carry FP32 rounding:
dH agrees to 5e-3 absolute, decisions where the margin exceeds 1e-2.
"""

import numpy as np
import pytest

import workloads as W
from oracle import hmc as OH
from oracle import philox as ph

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1103_4887_amd")

pytestmark = pytest.mark.gpu

MINV = np.array([0.3, 1e-5, 1e-5, 1e-5] + [1.0] * 7)


@pytest.fixture(scope="module")
def ctx():
    c = P.Context(0)
    yield c
    c.close()


def _chains(Ms, mask=0x7F, seed0=300):
    probs = []
    for i, M in enumerate(Ms):
        spec = W.ModelSpec(p_mask=mask)
        pr = W.make_hh_problem(M, 0.02, seed0 + i, model=spec, require_spike=False, init="truth")
        probs.append(pr)
    return probs


def _minv_p(probs):
    return (1e-3 * np.abs(np.asarray(W.P_STAR))) ** 2


def _oracle(probs, chains, seed, k0, eps, L, minv, n):
    outs = []
    for pr, chn in zip(probs, chains):
        X, p = pr.X0.copy(), pr.p0.copy()
        dHs, oks, us = [], [], []
        for k in range(k0, k0 + n):
            X, p, ok, dH = OH.hmc_proposal(pr.model, X, p, pr.y, pr.I, seed=seed, chain=chn, k=k, e=eps, L=L,
                                           minv_state=minv[:4], minv_param=minv[4:])
            dHs.append(dH)
            oks.append(ok)
            us.append(float(ph.uniform_open(ph.draw(seed, chn, 0, k, ph.TAG_HACC)[0, 0])))
        outs.append((X, p, np.array(dHs), np.array(oks), np.array(us)))
    return outs


@pytest.mark.parametrize("n", [1, 4])
def test_hmc_fp64_matches_oracle(ctx, n):
    probs = _chains([37, 300, 64])
    minv = MINV.copy()
    minv[4:] = _minv_p(probs)
    chains = [3, 8, 11]
    eps, L, seed, k0 = 0.004, 6, 77, 10
    batch = P.PackedBatch.pack([q.X0 for q in probs], [q.p0 for q in probs], [q.y for q in probs],
                               [q.I for q in probs], chains, "fp64")
    st = P.HmcStats.allocate(len(probs), n)
    print(f"hmc fp64 n={n}", flush=True)
    P.pimc_hmc(ctx, probs[0].model, batch, seed=seed, k0=k0, eps=eps, L_steps=L, minv=minv, n_proposals=n, stats=st)
    assert ctx.sync() == 0
    ref = _oracle(probs, chains, seed, k0, eps, L, minv, n)
    gdH = st.dH.cpu().numpy()
    acc = st.acc.cpu().numpy()
    for i, (Xo, po, dHo, oko, uo) in enumerate(ref):
        inside = np.isfinite(dHo)          # the oracle reports NaN for invalid trajectories
        np.testing.assert_allclose(gdH[i][inside], dHo[inside], rtol=1e-8, atol=1e-9)
        assert acc[i, 1] == (~inside).sum()
        safe = np.abs(dHo[inside] + np.log(uo[inside])) > 1e-6
        assert safe.all()   # this case is chosen away from ties
        assert acc[i, 0] == oko.sum()
        Xb, pb, _, _ = batch.window(i)
        np.testing.assert_allclose(Xb.cpu().numpy(), Xo, rtol=1e-10, atol=1e-10)
        np.testing.assert_allclose(pb.cpu().numpy(), po, rtol=1e-12)
    assert 0 < acc[:, 0].sum()


def test_hmc_fp32_close_to_oracle(ctx):
    probs = _chains([300, 129])
    minv = MINV.copy()
    minv[4:] = _minv_p(probs)
    chains = [1, 2]
    eps, L, seed, k0 = 0.004, 6, 5, 0
    batch = P.PackedBatch.pack([q.X0 for q in probs], [q.p0 for q in probs], [q.y for q in probs],
                               [q.I for q in probs], chains, "fp32")
    st = P.HmcStats.allocate(len(probs), 1)
    P.pimc_hmc(ctx, probs[0].model, batch, seed=seed, k0=k0, eps=eps, L_steps=L, minv=minv, n_proposals=1, stats=st)
    assert ctx.sync() == 0
    ref = _oracle(probs, chains, seed, k0, eps, L, minv, 1)
    gdH = st.dH.cpu().numpy()[:, 0]
    for i, (Xo, po, dHo, oko, uo) in enumerate(ref):
        assert abs(gdH[i] - dHo[0]) < 5e-3 + 1e-3 * abs(dHo[0])
        if abs(dHo[0] + np.log(uo[0])) > 1e-2:
            assert st.acc.cpu().numpy()[i, 0] == int(oko[0])


def test_hmc_fp64_reflection_matches_oracle(ctx):
    """Trajectories that cross the gate walls (m within 1e-3 of 1 at the spike
    peak, gate momenta large): reflections happen and the proposal equals the
    oracle's."""
    pr = W.make_hh_problem(400, 0.02, 101, model=W.ModelSpec(p_mask=0x7F), init="truth")
    minv = np.array([2.5e-3, 1e-4, 1e-4, 1e-4] + list((1e-3 * np.abs(pr.p0)) ** 2))
    eps, L, seed, k0, n = 0.006, 10, 5, 0, 3
    cnt = [0]
    r, rp, mask = OH.momenta(pr.model, seed, 2, k0, pr.M, minv[:4], minv[4:])
    OH.leapfrog(pr.model, pr.X0, pr.p0, pr.y, pr.I, r, rp, mask, eps, L, minv[:4], minv[4:], count=cnt)
    assert cnt[0] > 0
    batch = P.PackedBatch.pack([pr.X0], [pr.p0], [pr.y], [pr.I], [2], "fp64")
    st = P.HmcStats.allocate(1, n)
    P.pimc_hmc(ctx, pr.model, batch, seed=seed, k0=k0, eps=eps, L_steps=L, minv=minv, n_proposals=n, stats=st)
    assert ctx.sync() == 0
    Xo, po, dHo, oko, uo = _oracle([pr], [2], seed, k0, eps, L, minv, n)[0]
    assert np.isfinite(dHo).all()
    np.testing.assert_allclose(st.dH.cpu().numpy()[0], dHo, rtol=1e-8, atol=1e-9)
    assert (np.abs(dHo + np.log(uo)) > 1e-6).all()
    acc = st.acc.cpu().numpy()[0]
    assert acc[0] == oko.sum() == 1 and acc[1] == 0
    np.testing.assert_allclose(batch.X.cpu().numpy(), Xo, rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(batch.p.cpu().numpy()[0], po, rtol=1e-12)


def test_hmc_invalid_trajectory_rejects(ctx):
    probs = _chains([64])
    minv = MINV.copy()
    minv[4:] = _minv_p(probs)
    batch = P.PackedBatch.pack([probs[0].X0], [probs[0].p0], [probs[0].y], [probs[0].I], [0], "fp32")
    X_before = batch.X.clone()
    p_before = batch.p.clone()
    st = P.HmcStats.allocate(1, 2)
    P.pimc_hmc(ctx, probs[0].model, batch, seed=1, k0=0, eps=5.0, L_steps=3, minv=minv, n_proposals=2, stats=st)
    assert ctx.sync() == 0
    acc = st.acc.cpu().numpy()[0]
    assert acc[0] == 0 and acc[1] == 2
    assert torch.equal(batch.X, X_before) and torch.equal(batch.p, p_before)


def test_hmc_graph_replays_equal_eager(ctx):
    """Proposals replayed from one captured graph equal kernel-by-kernel
    proposals, including across two calls with eager work in between."""
    probs = _chains([300, 64])
    minv = MINV.copy()
    minv[4:] = _minv_p(probs)
    chains = [4, 9]

    def batch():
        return P.PackedBatch.pack([q.X0 for q in probs], [q.p0 for q in probs], [q.y for q in probs],
                                  [q.I for q in probs], chains, "fp32")

    ga = batch()
    sa1 = P.HmcStats.allocate(2, 3)
    sa2 = P.HmcStats.allocate(2, 3)
    P.pimc_hmc(ctx, probs[0].model, ga, seed=6, k0=0, eps=0.004, L_steps=5, minv=minv, n_proposals=3, stats=sa1)
    junk = torch.randn(4096, device="cuda")
    junk = (junk * junk).sum()
    torch.cuda.synchronize()
    P.pimc_hmc(ctx, probs[0].model, ga, seed=6, k0=3, eps=0.004, L_steps=5, minv=minv, n_proposals=3, stats=sa2)
    assert ctx.sync() == 0
    gb = batch()
    dHb = []
    for k in range(6):
        sb = P.HmcStats.allocate(2, 1)
        P.pimc_hmc(ctx, probs[0].model, gb, seed=6, k0=k, eps=0.004, L_steps=5, minv=minv, n_proposals=1, stats=sb)
        assert ctx.sync() == 0
        dHb.append(sb.dH.cpu().numpy()[:, 0])
    assert torch.equal(ga.X, gb.X) and torch.equal(ga.p, gb.p)
    dHa = np.concatenate([sa1.dH.cpu().numpy(), sa2.dH.cpu().numpy()], axis=1)
    np.testing.assert_array_equal(dHa, np.stack(dHb, axis=1))
