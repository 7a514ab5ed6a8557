"""Parity at the benchmark configurations' full sizes, in the launch
shapes the benchmark uses, on outputs the oracle can reproduce:

* the FP64 window of 256 steps (conductances sampled): a whole 2000-sweep
  chain with its statistics, in lockstep with the oracle;
* the 4096-step FP32 window in the benchmark shape (16 tiles of 128 threads
  x 2 sites): every site's proposal, action change and decision of one
  sweep (the same checks as the FP32 site parity at smaller sizes);
* the 512-window uneven batch: sampled windows of one batched launch equal
  their own single-window runs (which the site-parity tests tie to the
  oracle);
* 64 HMC chains of 16384 steps: sampled chains' energy changes and decisions
  against the oracle's leapfrog.
"""

import numpy as np
import pytest

import workloads as W
from oracle import hmc as OH
from oracle import philox as ph
from oracle import sampler as OS

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1103_4887_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = P.Context(0)
    yield c
    c.close()


def test_fp64_m256_full_chain_lockstep(ctx):
    c = W.CONFIGS["c1"]
    prob = W.config_problem("c1", init="truth", require_spike=False)
    n, burn = c["sweeps"], c["burn"]
    X, p = prob.X0.copy(), prob.p0.copy()
    st = OS.Stats(prob.M, 4, 7, n, burn=burn, xref=prob.X0.copy(), nbatch=32)
    print("oracle c1 chain", flush=True)
    OS.run(prob.model, X, p, prob.y, prob.I, seed=prob.seed, chain=1, sweep0=0, n_sweeps=n,
           w_state=prob.w_state, w_param=prob.w_param, stats=st)
    win = P.Window.from_arrays(prob.X0, prob.p0, prob.y, prob.I, "fp64")
    gst = P.SweepStats.allocate(win, n, burn=burn, nbatch=32)
    w = P.widths_tensor(prob.w_state, prob.w_param)
    print("gpu c1 chain", flush=True)
    P.pimc_sweep(ctx, prob.model, win, seed=prob.seed, chain=1, sweep0=0, w=w, n_sweeps=n, stats=gst)
    assert ctx.sync() == 0
    np.testing.assert_array_equal(gst.acc.cpu().numpy(), st.acc)
    np.testing.assert_allclose(win.X.cpu().numpy(), X, rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(win.p.cpu().numpy(), p, rtol=1e-12)
    np.testing.assert_allclose(gst.ptrace.cpu().numpy(), st.ptrace, rtol=1e-12)
    # posterior means and variances of the states (sums over the second half)
    np.testing.assert_allclose(gst.sum.cpu().numpy(), st.sum, rtol=1e-8, atol=1e-8)
    np.testing.assert_allclose(gst.sumsq.cpu().numpy(), st.sumsq, rtol=1e-8, atol=1e-10)
    # batch means (32 runs of consecutive samples) for the MCSE of the path means
    np.testing.assert_allclose(gst.batch.cpu().numpy(), st.batch, rtol=1e-8, atol=1e-8)


def test_c4_batch_sampled_windows_equal_single_runs(ctx):
    probs = W.config_batch("c4", workers=8)
    spec = probs[0].model
    B = len(probs)
    chains = list(range(B))
    batch = P.PackedBatch.pack([q.X0 for q in probs], [q.p0 for q in probs], [q.y for q in probs],
                               [q.I for q in probs], chains, "fp32")
    w = P.widths_tensor(probs[0].w_state, probs[0].w_param)
    n = 3
    print(f"c4 batch of {B} windows, {int(batch.offsets[-1])} sites", flush=True)
    P.pimc_run_batch(ctx, spec, batch, seed=104, sweep0=0, w=w, n_sweeps=n)
    assert ctx.sync() == 0
    sizes = np.diff(batch.offsets)
    picks = sorted({int(np.argmax(sizes)), int(np.argmin(sizes)), 0, B // 3, B // 2, B - 1})
    for i in picks:
        q = probs[i]
        win = P.Window.from_arrays(q.X0, q.p0, q.y, q.I, "fp32")
        P.pimc_sweep(ctx, spec, win, seed=104, chain=chains[i], sweep0=0, w=w, n_sweeps=n)
        assert ctx.sync() == 0
        Xb, pb, _, _ = batch.window(i)
        np.testing.assert_array_equal(Xb.cpu().numpy(), win.X.cpu().numpy())
        np.testing.assert_allclose(pb.cpu().numpy(), win.p.cpu().numpy(), rtol=1e-14)


def test_c5_hmc_sampled_chains_match_oracle(ctx):
    c = W.CONFIGS["c5"]
    prob = W.config_problem("c5", init="truth", require_spike=False)
    B = c["chains"]
    minv = np.array([0.05, 1e-5, 1e-5, 1e-5] + list((1e-3 * np.abs(prob.p0)) ** 2))
    eps, L, seed, k0 = 0.004, c["leapfrog"], 105, 0
    batch = P.PackedBatch.pack([prob.X0] * B, [prob.p0] * B, [prob.y] * B, [prob.I] * B, list(range(B)), "fp32")
    st = P.HmcStats.allocate(B, 1)
    print("gpu c5 hmc", flush=True)
    P.pimc_hmc(ctx, prob.model, batch, seed=seed, k0=k0, eps=eps, L_steps=L, minv=minv, n_proposals=1, stats=st)
    assert ctx.sync() == 0
    gdH = st.dH.cpu().numpy()[:, 0]
    gacc = st.acc.cpu().numpy()[:, 0]
    X32 = prob.X0.astype(np.float32).astype(np.float64)
    y32 = prob.y.astype(np.float32).astype(np.float64)
    I32 = prob.I.astype(np.float32).astype(np.float64)
    for chn in (0, B - 1):
        print(f"oracle c5 chain {chn}", flush=True)
        _, _, ok, dH = OH.hmc_proposal(prob.model, X32, prob.p0, y32, I32, seed=seed, chain=chn, k=k0, e=eps, L=L,
                                       minv_state=minv[:4], minv_param=minv[4:])
        assert np.isfinite(dH)
        # the FP32 trajectory's rounding adds up like a random walk over the
        # coordinates: 5e-3 at 300 sites (the small-window FP32 test) scaled by
        # the square root of the site count
        tol = 5e-3 * np.sqrt((prob.M + 1) / 300.0) + 1e-3 * abs(dH)
        assert abs(gdH[chn] - dH) < tol, (chn, gdH[chn], dH, tol)
        u = float(ph.uniform_open(ph.draw(seed, chn, 0, k0, ph.TAG_HACC)[0, 0]))
        if abs(dH + np.log(u)) > 2 * tol:
            assert gacc[chn] == int(ok)
