"""Exact conditional parameter draws (PIMC_GIBBS) of the HIP library against
the oracle (oracle/gibbs.py).

The library reads each conditional from its path statistics (s, G); the
oracle fits the quadratic of the direct-sum action over the box; both invert
the truncated normal CDF with the same uniform.  FP64 chains run in lockstep
(whole sweeps: sites, then the seven draws); in FP32 mode the draws of one
sweep at the benchmark's tiled launch shape are compared with the oracle's
draws on the GPU's own path.  Bars: drawn values within 1e-9 relative (both
sides form the conditional in FP64), paths within 1e-9.
"""

import numpy as np
import pytest

import workloads as W
from oracle import gibbs as OG
from oracle import sampler as OS

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1103_4887_amd")

pytestmark = pytest.mark.gpu

GIBBS = 4


@pytest.fixture(scope="module")
def ctx():
    c = P.Context(0)
    yield c
    c.close()


def test_gibbs_fp64_lockstep(ctx):
    spec = W.ModelSpec(p_mask=0x7F)
    prob = W.make_hh_problem(300, 0.02, 131, model=spec, require_spike=False, init="guess")
    n = 6
    X, p = prob.X0.copy(), prob.p0.copy()
    st = OS.Stats(prob.M, 4, 7, n)
    od = OS.Debug()
    OS.run(spec, X, p, prob.y, prob.I, seed=prob.seed, chain=4, sweep0=20, n_sweeps=n, w_state=prob.w_state,
           w_param=prob.w_param, flags=OS.STATES | OS.PARAMS | OS.GIBBS, stats=st, debug=od)
    ctx.set_tiles(0)
    win = P.Window.from_arrays(prob.X0, prob.p0, prob.y, prob.I, "fp64")
    gst = P.SweepStats.allocate(win, n, moments=False)
    gd = P.SweepDebug.allocate(win, sites=False, params=True)
    w = P.widths_tensor(prob.w_state, prob.w_param)
    print("gibbs fp64 lockstep M=300", flush=True)
    P.pimc_sweep(ctx, spec, win, seed=prob.seed, chain=4, sweep0=20, w=w, n_sweeps=n,
                 flags=P._lib.PIMC_STATES | P._lib.PIMC_PARAMS | GIBBS, stats=gst, debug=gd)
    assert ctx.sync() == 0
    np.testing.assert_allclose(gst.ptrace.cpu().numpy(), st.ptrace, rtol=1e-9)
    np.testing.assert_allclose(gd.pprop.cpu().numpy(), od.pprop, rtol=1e-9)
    np.testing.assert_array_equal(gd.paccept.cpu().numpy().astype(bool), od.paccept)
    np.testing.assert_allclose(win.X.cpu().numpy(), X, rtol=1e-9, atol=1e-9)
    acc = gst.acc.cpu().numpy()
    np.testing.assert_array_equal(acc[2:9], st.acc[2:9])       # every draw finite, counted
    assert (acc[2:9] == n).all()


@pytest.mark.parametrize("K,T", [
    (2, 16),
    pytest.param(0, 0, marks=pytest.mark.skip(
        reason="a GPU run of this case (then 16 sites x 256 threads, one workgroup, extended kernel) was "
               "followed by a GPU fault whose cause is not identified; the extended kernels no longer take that "
               "shape, and the case stays off the GPU until the cause is known")),
])
def test_gibbs_fp32_draws_match_oracle_on_gpu_path(ctx, K, T):
    prob = W.config_problem("c2", init="guess")
    spec = prob.model
    ctx.set_tile(K)
    ctx.set_tiles(T)
    try:
        win = P.Window.from_arrays(prob.X0, prob.p0, prob.y, prob.I, "fp32")
        w = P.widths_tensor(prob.w_state, prob.w_param)
        gd = P.SweepDebug.allocate(win, sites=False, params=True)
        print(f"gibbs fp32 one sweep M={prob.M} K={K} T={T}", flush=True)
        P.pimc_sweep(ctx, spec, win, seed=prob.seed, chain=0, sweep0=55, w=w, n_sweeps=1,
                     flags=P._lib.PIMC_STATES | P._lib.PIMC_PARAMS | GIBBS, debug=gd)
        assert ctx.sync() == 0
    finally:
        ctx.set_tile(0)
        ctx.set_tiles(0)
    Xg = win.X.cpu().numpy().astype(np.float64)
    I32 = prob.I.astype(np.float32).astype(np.float64)
    p = prob.p0.astype(np.float64).copy()
    OG.param_gibbs(spec, Xg, I32, p, 55, prob.seed, 0)
    np.testing.assert_allclose(gd.pprop.cpu().numpy(), p, rtol=1e-9)
    np.testing.assert_allclose(win.p.cpu().numpy(), p, rtol=1e-9)


def test_extended_kernels_refused_at_sixteen_sites_per_thread(ctx):
    """16 sites per thread is refused on the host for the extended kernels
    (exact draws, initialization phase, Table 1 constants): nothing is
    launched and the path is unchanged."""
    prob = W.config_problem("c2", init="guess")
    win = P.Window.from_arrays(prob.X0, prob.p0, prob.y, prob.I, "fp32")
    w = P.widths_tensor(prob.w_state, prob.w_param)
    X0 = win.X.clone()
    ctx.set_tile(16)
    ctx.set_tiles(1)
    try:
        with pytest.raises(P._lib.PimcError) as e:
            P.pimc_sweep(ctx, prob.model, win, seed=prob.seed, chain=0, sweep0=1, w=w, n_sweeps=1,
                         flags=P._lib.PIMC_STATES | P._lib.PIMC_PARAMS | GIBBS)
        assert e.value.status == P._lib.PIMC_ERR_UNSUPPORTED
        gi = P.InitPhase.start(win, prob.w_param, beta0=0.5, n_cool=4, n_init=4, n_skip=2)
        with pytest.raises(P._lib.PimcError) as e:
            P.pimc_sweep_init(ctx, prob.model, win, seed=prob.seed, chain=0, sweep0=1, w=w, n_sweeps=1, init=gi)
        assert e.value.status == P._lib.PIMC_ERR_UNSUPPORTED
    finally:
        ctx.set_tile(0)
        ctx.set_tiles(0)
    assert ctx.sync() == 0
    assert torch.equal(win.X, X0)


def test_gibbs_tiled_batch_equals_single_runs(ctx):
    """Exact draws inside a batch of windows cut into time tiles (the launch
    of the batched comparison: 8 tiles of 256 threads x 2 sites for M = 4096)
    give each window exactly the chain of its own single-window run at the
    same tiling: equal paths, parameters within the rounding of the
    cross-tile sums."""
    probs = [W.make_hh_problem(4096, 0.02, 190 + i, require_spike=False, init="truth") for i in range(3)]
    spec = probs[0].model
    chains = [11, 12, 13]
    w = P.widths_tensor(probs[0].w_state, probs[0].w_param)
    flags = P._lib.PIMC_STATES | P._lib.PIMC_PARAMS | GIBBS
    batch = P.PackedBatch.pack([q.X0 for q in probs], [q.p0 for q in probs], [q.y for q in probs],
                               [q.I for q in probs], chains, "fp32")
    ctx.set_tile(2)
    ctx.set_tiles(8)
    try:
        print("gibbs tiled batch of 3 windows M=4096, 8 tiles", flush=True)
        P.pimc_run_batch(ctx, spec, batch, seed=6, sweep0=40, w=w, n_sweeps=12, flags=flags)
        assert ctx.sync() == 0
        for i, q in enumerate(probs):
            win = P.Window.from_arrays(q.X0, q.p0, q.y, q.I, "fp32")
            P.pimc_sweep(ctx, spec, win, seed=6, chain=chains[i], sweep0=40, w=w, n_sweeps=12, flags=flags)
            assert ctx.sync() == 0
            Xb, pb, _, _ = batch.window(i)
            np.testing.assert_array_equal(Xb.cpu().numpy(), win.X.cpu().numpy())
            np.testing.assert_allclose(pb.cpu().numpy(), win.p.cpu().numpy(), rtol=1e-13)
            assert not np.array_equal(pb.cpu().numpy(), q.p0)      # the draws moved the parameters
    finally:
        ctx.set_tile(0)
        ctx.set_tiles(0)
