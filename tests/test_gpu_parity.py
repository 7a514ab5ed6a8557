"""Parity of the HIP library (through its C ABI) with the CPU oracle.

Tolerances (written per test):
  * FP64 site arithmetic: per-site dA within 1e-12 * max(1, |dA|) of the
    oracle's, accept decisions identical wherever |dA + log u| > 1e-6;
  * FP32 site arithmetic: dA evaluated by the oracle on the GPU's own
    proposal within 1e-4 * max(1, |dA|); decisions identical wherever
    |dA + log u| > 1e-4 * max(1, |dA|);
  * action: FP64 terms in both precisions -> 1e-12 relative;
  * parameter moves: the GPU's sufficient-statistic dA equals the oracle's
    direct sum over the path to 1e-9 relative (FP64 sums on both sides);
  * integer work (acceptance counters, decisions away from ties): exact.
"""

import numpy as np
import pytest

import workloads as W
from oracle import action as OA
from oracle import sampler as OS

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1103_4887_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = P.Context(0)
    yield c
    c.close()


def _problem(M, seed=101, init="guess", mask=0x7F, proposal="gauss", dt=0.02):
    spec = W.ModelSpec(dt=dt, p_mask=mask, proposal=proposal)
    prob = W.make_hh_problem(M, dt, seed, model=spec, require_spike=False, init=init)
    return prob


def _perturbed(prob, seed=0):
    """A state off the truth (a realistic mid-run path), inside the box."""
    rng = np.random.default_rng(seed)
    X = prob.X_true + rng.normal(size=prob.X_true.shape) * np.array([0.3, 2e-3, 2e-3, 2e-3])
    X[:, 1:] = np.clip(X[:, 1:], 0.0, 1.0)
    return X


def _oracle_one_sweep(prob, X, p, sweep, chain=0, flags=3):
    X = X.copy()
    p = p.copy()
    dbg = OS.Debug()
    st = OS.Stats(prob.M, 4, 7, 1)
    OS.run(prob.model, X, p, prob.y, prob.I, seed=prob.seed, chain=chain, sweep0=sweep, n_sweeps=1,
           w_state=prob.w_state, w_param=prob.w_param, flags=flags, stats=st, debug=dbg)
    return X, p, dbg, st


def _gpu_one_sweep(ctx, prob, X, p, sweep, prec, chain=0, flags=3, tiles=0):
    ctx.set_tiles(tiles)
    win = P.Window.from_arrays(X, p, prob.y, prob.I, prec)
    w = P.widths_tensor(prob.w_state, prob.w_param)
    dbg = P.SweepDebug.allocate(win)
    st = P.SweepStats.allocate(win, 1, moments=False)
    print(f"gpu sweep prec={prec} M={prob.M} sweep={sweep} flags={flags} tiles={tiles}", flush=True)
    P.pimc_sweep(ctx, prob.model, win, seed=prob.seed, chain=chain, sweep0=sweep, w=w, n_sweeps=1,
                 flags=flags, stats=st, debug=dbg)
    rc = ctx.sync()
    ctx.set_tiles(0)
    assert rc == 0
    return win, dbg, st


@pytest.mark.parametrize("M", [1, 2, 7, 8, 9, 37, 256, 300])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_action_matches_oracle(ctx, M, prec):
    prob = _problem(M)
    X = _perturbed(prob)
    if prec == "fp32":
        X = X.astype(np.float32).astype(np.float64)
    spec = prob.model.with_(beta=0.7)
    win = P.Window.from_arrays(X, prob.p0, prob.y, prob.I, prec)
    out = P.pimc_action(ctx, spec, win).cpu().numpy()
    y = prob.y.astype(np.float32).astype(np.float64) if prec == "fp32" else prob.y
    I = prob.I.astype(np.float32).astype(np.float64) if prec == "fp32" else prob.I
    ref = OA.action(spec, X, y, I, prob.p0)
    np.testing.assert_allclose(out, ref, rtol=1e-12)


@pytest.mark.parametrize("M", [1, 5, 255, 256, 300])
def test_grad_matches_oracle_fp64(ctx, M):
    prob = _problem(M)
    X = _perturbed(prob, 1)
    spec = prob.model.with_(beta=0.9)
    win = P.Window.from_arrays(X, prob.p0, prob.y, prob.I, "fp64")
    gX, gp = P.pimc_grad(ctx, spec, win)
    g_ref, gp_ref = OA.grad(spec, X, prob.y, prob.I, prob.p0)
    scale = np.abs(g_ref).max()
    np.testing.assert_allclose(gX.cpu().numpy(), g_ref, rtol=1e-10, atol=1e-12 * scale)
    np.testing.assert_allclose(gp.cpu().numpy(), gp_ref, rtol=1e-9, atol=1e-12 * np.abs(gp_ref).max())


@pytest.mark.parametrize("M", [300, 4096])
def test_grad_fp32_within_rounding_bound(ctx, M):
    """Every entry of the FP32 gradient lies within its first-order FP32
    rounding bound (tests/fp32_bounds.py) of the FP64 oracle's gradient on
    the same FP32 inputs; no entry is exempt."""
    import fp32_bounds as FB
    prob = _problem(M)
    X = _perturbed(prob, 2).astype(np.float32).astype(np.float64)
    win = P.Window.from_arrays(X, prob.p0, prob.y, prob.I, "fp32")
    gX, gp = P.pimc_grad(ctx, prob.model, win)
    y32 = prob.y.astype(np.float32).astype(np.float64)
    I32 = prob.I.astype(np.float32).astype(np.float64)
    g_ref, gp_ref = OA.grad(prob.model, X, y32, I32, prob.p0)
    bound, gp_bound = FB.grad_bound(prob.model, X, y32, I32, prob.p0)
    err = np.abs(gX.cpu().numpy().astype(np.float64) - g_ref)
    ratio = err / bound
    print(f"grad fp32 M={M}: max error / bound {ratio.max():.3g}, median {np.median(ratio):.3g}")
    assert (err <= bound).all(), np.unravel_index(np.argmax(ratio), ratio.shape)
    gerr = np.abs(gp.cpu().numpy() - gp_ref)
    assert (gerr <= gp_bound).all(), gerr / gp_bound


def _check_sites(gdbg, odbg, tol, margin_of):
    gdA = gdbg.dA.cpu().numpy()
    gacc = gdbg.accept.cpu().numpy().astype(bool)
    fin_g = np.isfinite(gdA)
    fin_o = np.isfinite(odbg.dA)
    assert np.array_equal(fin_g, fin_o), np.nonzero(fin_g != fin_o)
    err = np.abs(gdA[fin_o] - odbg.dA[fin_o]) / np.maximum(1.0, np.abs(odbg.dA[fin_o]))
    assert err.max() <= tol, err.max()
    margin = np.abs(odbg.dA + np.log(odbg.u))
    safe = ~fin_o | (margin > margin_of(odbg.dA))
    assert np.array_equal(gacc[safe], odbg.accept[safe])
    return int((~safe).sum())


FP64_WIDE_OFF = pytest.mark.skip(
    reason="FP64 windows above 1024 sites are refused: the wide FP64 shapes (more than 256 threads) spill about "
           "1 KB per thread and the 8 x 512 shape faulted the GPU once (M = 4096) without an identified cause")
FP64_TILES_OFF = pytest.mark.skip(
    reason="FP64 time tiles are switched off: a 16-tile FP64 window faulted the GPU once (memory aperture "
           "violation) and no cause has been shown yet; the library refuses FP64 tiled shapes")


@pytest.mark.parametrize("M,tiles", [(1, 0), (2, 0), (8, 0), (9, 0), (37, 0), (256, 0), (300, 0), (1000, 0),
                                     (1024, 0),
                                     pytest.param(4096, 0, marks=FP64_WIDE_OFF),
                                     pytest.param(1000, 2, marks=FP64_TILES_OFF),
                                     pytest.param(1000, 4, marks=FP64_TILES_OFF),
                                     pytest.param(4096, 16, marks=FP64_TILES_OFF),
                                     pytest.param(2049, 9, marks=FP64_TILES_OFF)])
def test_sweep_fp64_lockstep(ctx, M, tiles):
    prob = _problem(M)
    X = _perturbed(prob, 3)
    p = prob.p_true * 1.01
    for sweep in (0, 12345678901):
        Xo, po, od, so = _oracle_one_sweep(prob, X, p, sweep)
        win, gd, gs = _gpu_one_sweep(ctx, prob, X, p, sweep, "fp64", tiles=tiles)
        np.testing.assert_allclose(gd.xprop.cpu().numpy(), od.xprop, rtol=1e-14, atol=1e-14)
        ties = _check_sites(gd, od, 1e-12, lambda d: 1e-6)
        gpdA = gd.pdA.cpu().numpy()
        m = np.isfinite(od.pdA)
        np.testing.assert_array_equal(np.isfinite(gpdA), m)
        np.testing.assert_allclose(gpdA[m], od.pdA[m], rtol=1e-9, atol=1e-9)
        np.testing.assert_allclose(gd.pprop.cpu().numpy()[m], od.pprop[m], rtol=1e-15)
        if ties == 0:
            np.testing.assert_allclose(win.X.cpu().numpy(), Xo, rtol=1e-13, atol=1e-13)
            np.testing.assert_allclose(win.p.cpu().numpy(), po, rtol=1e-14)
            np.testing.assert_array_equal(gs.acc.cpu().numpy(), so.acc)


@pytest.mark.parametrize("M,tiles,K", [(8, 0, 0), (37, 0, 0), (256, 0, 0), (4096, 0, 0), (8192, 0, 0), (4096, 4, 0),
                                       (65536, 0, 0), (37, 0, 2), (510, 0, 2), (4096, 8, 2), (4095, 8, 2),
                                       (4094, 8, 2), (4096, 16, 2)])
def test_sweep_fp32_site_parity(ctx, M, tiles, K):
    prob = _problem(M, dt=0.01 if M > 8192 else 0.02)
    X = _perturbed(prob, 4).astype(np.float32).astype(np.float64)
    p = prob.p_true * 0.99
    y32 = prob.y.astype(np.float32).astype(np.float64)
    I32 = prob.I.astype(np.float32).astype(np.float64)
    ctx.set_tile(K)
    try:
        win, gd, gs = _gpu_one_sweep(ctx, prob, X, p, 77, "fp32", flags=P._lib.PIMC_STATES, tiles=tiles)
    finally:
        ctx.set_tile(0)
    xp = gd.xprop.cpu().numpy().astype(np.float64)
    # proposals: same Philox words, FP32 Box-Muller vs FP64
    Xo, po, od, so = _oracle_one_sweep(prob, X, p, 77, flags=OS.STATES)
    np.testing.assert_allclose(xp, od.xprop, rtol=2e-6, atol=2e-6 * np.abs(prob.w_state).max() * 10)
    # dA of the GPU's own proposal, re-evaluated by the oracle on the same state
    M1 = prob.M + 1
    gdA = gd.dA.cpu().numpy()
    gacc = gd.accept.cpu().numpy().astype(bool)
    ref = np.full(M1, np.nan)
    lo, hi = np.asarray(prob.model.x_lo), np.asarray(prob.model.x_hi)
    Xcur = X.copy()
    for color in (0, 1):
        ns = np.arange(color, M1, 2)
        inb = ((xp[ns] >= lo) & (xp[ns] <= hi)).all(axis=1)
        d = np.full(len(ns), np.nan)
        if inb.any():
            d[inb] = OA.delta_site(prob.model, Xcur, y32, I32, p, ns[inb], xp[ns][inb])
        ref[ns] = d
        acc_n = ns[gacc[ns]]
        Xcur[acc_n] = xp[acc_n]
    fin = np.isfinite(ref)
    np.testing.assert_array_equal(np.isfinite(gdA), fin)
    err = np.abs(gdA[fin] - ref[fin]) / np.maximum(1.0, np.abs(ref[fin]))
    assert err.max() <= 1e-4, err.max()
    u = od.u
    margin = np.abs(ref + np.log(u))
    safe = fin & (margin > 1e-4 * np.maximum(1.0, np.abs(ref)))
    decide = np.log(u) < -ref
    np.testing.assert_array_equal(gacc[safe], decide[safe])
    assert not gacc[~fin].any()
    np.testing.assert_allclose(win.X.cpu().numpy().astype(np.float64), Xcur, rtol=0, atol=0)


def test_param_moves_fp32_match_direct_sum(ctx):
    prob = _problem(4096)
    X = _perturbed(prob, 5).astype(np.float32).astype(np.float64)
    p = prob.p_true * 1.02
    I32 = prob.I.astype(np.float32).astype(np.float64)
    win, gd, gs = _gpu_one_sweep(ctx, prob, X, p, 5, "fp32", flags=P._lib.PIMC_PARAMS)
    gpdA = gd.pdA.cpu().numpy()
    gpprop = gd.pprop.cpu().numpy()
    gacc = gd.paccept.cpu().numpy().astype(bool)
    cur = p.copy()
    for l in range(7):
        pp = cur.copy()
        pp[l] = gpprop[l]
        ref = OA.delta_params(prob.model, X, I32, cur, pp)
        assert gpdA[l] == pytest.approx(ref, rel=1e-9, abs=1e-9), l
        if gacc[l]:
            cur = pp
    np.testing.assert_allclose(win.p.cpu().numpy(), cur, rtol=1e-15)


@pytest.mark.parametrize("K,T", [(2, 128), (0, 64)])
def test_param_moves_long_window_tiled_match_direct_sum(ctx, K, T):
    """The M = 65536 window (dt = 0.01 ms) in its tiled launch shapes (128
    tiles of 128 threads x 2 sites; 64 tiles of 256 x 4): after a full sweep
    (sites, then the seven moves against the parameter statistics summed
    over all tiles), each move's dA equals the oracle's direct sum over the
    GPU's path to 1e-9, and each decision is log u < -dA with the oracle's u
    wherever the margin exceeds 1e-6."""
    prob = W.config_problem("c3")
    X = _perturbed(prob, 6).astype(np.float32).astype(np.float64)
    p = prob.p_true * 1.01
    I32 = prob.I.astype(np.float32).astype(np.float64)
    ctx.set_tile(K)
    try:
        win, gd, gs = _gpu_one_sweep(ctx, prob, X, p, 77, "fp32", flags=3, tiles=T)
    finally:
        ctx.set_tile(0)
        ctx.set_tiles(0)
    Xg = win.X.cpu().numpy().astype(np.float64)     # the path the moves saw
    gpdA = gd.pdA.cpu().numpy()
    gpprop = gd.pprop.cpu().numpy()
    gacc = gd.paccept.cpu().numpy().astype(bool)
    # the oracle's accept uniforms of this sweep's parameter moves
    _, _, od, _ = _oracle_one_sweep(prob, Xg, p, 77, flags=OS.PARAMS)
    cur = p.copy()
    for l in range(7):
        pp = cur.copy()
        pp[l] = gpprop[l]
        ref = OA.delta_params(prob.model, Xg, I32, cur, pp)
        assert gpdA[l] == pytest.approx(ref, rel=1e-9, abs=1e-9), l
        if abs(ref + np.log(od.pu[l])) > 1e-6:
            assert gacc[l] == (np.log(od.pu[l]) < -ref), l
        if gacc[l]:
            cur = pp
    np.testing.assert_allclose(win.p.cpu().numpy(), cur, rtol=1e-15)


def test_multi_sweep_fp64_chain_and_stats(ctx):
    prob = _problem(300, init="guess", mask=W.configs.MASK_C1)
    n = 40
    X, p = prob.X0.copy(), prob.p0.copy()
    # samples after sweeps 110, 114, .., 138 (eight), in batches of 3, 3, 2
    st = OS.Stats(prob.M, 4, 7, n, burn=110, xref=prob.X0.copy(), stride=4, nbatch=3)
    OS.run(prob.model, X, p, prob.y, prob.I, seed=prob.seed, chain=3, sweep0=100, n_sweeps=n,
           w_state=prob.w_state, w_param=prob.w_param, stats=st)
    win = P.Window.from_arrays(prob.X0, prob.p0, prob.y, prob.I, "fp64")
    gst = P.SweepStats.allocate(win, n, burn=110, stride=4, nbatch=3)
    w = P.widths_tensor(prob.w_state, prob.w_param)
    P.pimc_sweep(ctx, prob.model, win, seed=prob.seed, chain=3, sweep0=100, w=w, n_sweeps=n, stats=gst)
    assert ctx.sync() == 0
    np.testing.assert_allclose(win.X.cpu().numpy(), X, rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(win.p.cpu().numpy(), p, rtol=1e-12)
    np.testing.assert_allclose(gst.ptrace.cpu().numpy(), st.ptrace, rtol=1e-12)
    np.testing.assert_allclose(gst.sum.cpu().numpy(), st.sum, rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(gst.sumsq.cpu().numpy(), st.sumsq, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(gst.batch.cpu().numpy(), st.batch, rtol=1e-9, atol=1e-9)
    np.testing.assert_array_equal(gst.acc.cpu().numpy(), st.acc)


@pytest.mark.parametrize("M,stride", [(8192, 1), (4096, 3), (37, 2)])
def test_moments_fp32_large_window(ctx, M, stride):
    """Moment sums (staged through LDS in chunks at large M) equal the sums
    of the chain's own states, sweep by sweep."""
    prob = _problem(M)
    win = P.Window.from_arrays(prob.X0, prob.p0, prob.y, prob.I, "fp32")
    w = P.widths_tensor(prob.w_state, prob.w_param)
    st = P.SweepStats.allocate(win, 1, burn=2, stride=stride)
    xref = st.xref.cpu().numpy().astype(np.float64)
    S = np.zeros((M + 1, 4))
    Q = np.zeros((M + 1, 4))
    for k in range(9):
        P.pimc_sweep(ctx, prob.model, win, seed=3, chain=0, sweep0=k, w=w, n_sweeps=1, stats=st)
        if k >= 2 and (k - 2) % stride == 0:
            d = win.X.cpu().numpy().astype(np.float64) - xref
            S += d
            Q += d * d
    assert ctx.sync() == 0
    np.testing.assert_allclose(st.sum.cpu().numpy(), S, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(st.sumsq.cpu().numpy(), Q, rtol=1e-12, atol=1e-15)


def test_tiling_invariance_fp32(ctx):
    prob = _problem(1000)
    w = P.widths_tensor(prob.w_state, prob.w_param)
    outs = []
    for K, T in ((4, 0), (8, 0), (16, 0), (2, 4)):
        ctx.set_tile(K)
        ctx.set_tiles(T)
        win = P.Window.from_arrays(prob.X0, prob.p0, prob.y, prob.I, "fp32")
        P.pimc_sweep(ctx, prob.model, win, seed=9, chain=1, sweep0=0, w=w, n_sweeps=25)
        assert ctx.sync() == 0
        outs.append((win.X.cpu().numpy(), win.p.cpu().numpy()))
    ctx.set_tile(0)
    ctx.set_tiles(0)
    for X, p in outs[1:]:
        np.testing.assert_array_equal(X, outs[0][0])
        np.testing.assert_allclose(p, outs[0][1], rtol=1e-14)


@pytest.mark.parametrize("M", [4096, 65536])
def test_time_tiles_give_the_same_chain(ctx, M):
    """Cutting the window into time tiles (halo exchange + cross-tile
    all-reduce) leaves the chain unchanged: site updates are bit-identical,
    parameter decisions equal (the reduction order differs only in rounding)."""
    prob = _problem(M, dt=0.01 if M > 8192 else 0.02)
    w = P.widths_tensor(prob.w_state, prob.w_param)
    outs = []
    choices = ((0, 1), (0, 2), (0, 4), (0, 16), (2, 8), (2, 16)) if M == 4096 else ((0, 0), (0, 32), (0, 64), (2, 128))
    n = 20 if M == 4096 else 4
    for K, T in choices:
        ctx.set_tile(K)
        ctx.set_tiles(T)
        win = P.Window.from_arrays(prob.X0, prob.p0, prob.y, prob.I, "fp32")
        st = P.SweepStats.allocate(win, n, burn=0)
        print(f"K={K} tiles={T} M={M}", flush=True)
        P.pimc_sweep(ctx, prob.model, win, seed=21, chain=2, sweep0=5, w=w, n_sweeps=n, stats=st)
        rc = ctx.sync()
        ctx.set_tiles(0)
        ctx.set_tile(0)
        assert rc == 0
        outs.append((win.X.cpu().numpy(), win.p.cpu().numpy(), st.acc.cpu().numpy(), st.sum.cpu().numpy(),
                     st.ptrace.cpu().numpy()))
    for X, p, acc, su, tr in outs[1:]:
        np.testing.assert_array_equal(X, outs[0][0])
        np.testing.assert_allclose(p, outs[0][1], rtol=1e-14)
        np.testing.assert_array_equal(acc, outs[0][2])
        np.testing.assert_allclose(su, outs[0][3], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(tr, outs[0][4], rtol=1e-14)


def test_batch_window_equals_single_run(ctx):
    Ms = [37, 300, 64, 129]
    probs = [W.make_hh_problem(M, 0.02, 200 + i, require_spike=False) for i, M in enumerate(Ms)]
    spec = probs[0].model
    chains = [5, 6, 7, 8]
    batch = P.PackedBatch.pack([q.X0 for q in probs], [q.p0 for q in probs], [q.y for q in probs],
                               [q.I for q in probs], chains, "fp32")
    w = P.widths_tensor(probs[0].w_state, probs[0].w_param)
    P.pimc_run_batch(ctx, spec, batch, seed=4, sweep0=10, w=w, n_sweeps=15)
    assert ctx.sync() == 0
    for i, q in enumerate(probs):
        win = P.Window.from_arrays(q.X0, q.p0, q.y, q.I, "fp32")
        P.pimc_sweep(ctx, spec, win, seed=4, chain=chains[i], sweep0=10, w=w, n_sweeps=15)
        assert ctx.sync() == 0
        Xb, pb, _, _ = batch.window(i)
        np.testing.assert_array_equal(Xb.cpu().numpy(), win.X.cpu().numpy())
        np.testing.assert_allclose(pb.cpu().numpy(), win.p.cpu().numpy(), rtol=1e-14)


@pytest.mark.parametrize("Ms,T", [([4096, 3500, 3073], 4), ([4096, 600, 2000], 4), ([8192, 8000], 8)])
def test_tiled_batch_equals_single_runs(ctx, Ms, T):
    """Windows that all need T tiles run tiled inside the batch (B x T
    workgroups); a ragged batch falls back to one workgroup per window.
    Either way every window's chain and statistics equal its own untiled
    run (tiling changes only the rounding of the parameter sums)."""
    probs = [W.make_hh_problem(M, 0.02, 400 + i, require_spike=False) for i, M in enumerate(Ms)]
    spec = probs[0].model
    chains = [11 + i for i in range(len(Ms))]
    w = P.widths_tensor(probs[0].w_state, probs[0].w_param)
    n = 12
    batch = P.PackedBatch.pack([q.X0 for q in probs], [q.p0 for q in probs], [q.y for q in probs],
                               [q.I for q in probs], chains, "fp32")
    dev = batch.X.device
    bst = P.SweepStats(sum=torch.zeros(batch.X.shape, dtype=torch.float64, device=dev),
                       sumsq=torch.zeros(batch.X.shape, dtype=torch.float64, device=dev), xref=batch.X.clone(),
                       ptrace=torch.zeros((len(Ms), n, 7), dtype=torch.float64, device=dev),
                       acc=torch.zeros((len(Ms), P._lib.PIMC_NACC), dtype=torch.int64, device=dev), burn=0,
                       batch=torch.zeros((5,) + tuple(batch.X.shape), dtype=torch.float64, device=dev))
    ctx.set_tiles(T)
    try:
        print(f"tiled batch Ms={Ms} T={T}", flush=True)
        P.pimc_run_batch(ctx, spec, batch, seed=8, sweep0=3, w=w, n_sweeps=n, stats=bst)
        assert ctx.sync() == 0
        for i, q in enumerate(probs):
            ctx.set_tiles(1)
            win = P.Window.from_arrays(q.X0, q.p0, q.y, q.I, "fp32")
            st = P.SweepStats.allocate(win, n, burn=0, nbatch=5)
            P.pimc_sweep(ctx, spec, win, seed=8, chain=chains[i], sweep0=3, w=w, n_sweeps=n, stats=st)
            assert ctx.sync() == 0
            a, b = int(batch.offsets[i]), int(batch.offsets[i + 1])
            np.testing.assert_array_equal(batch.X[a:b].cpu().numpy(), win.X.cpu().numpy())
            np.testing.assert_allclose(batch.p[i].cpu().numpy(), win.p.cpu().numpy(), rtol=1e-14)
            np.testing.assert_array_equal(bst.acc[i].cpu().numpy(), st.acc.cpu().numpy())
            np.testing.assert_allclose(bst.ptrace[i].cpu().numpy(), st.ptrace.cpu().numpy(), rtol=1e-14)
            np.testing.assert_allclose(bst.sum[a:b].cpu().numpy(), st.sum.cpu().numpy(), rtol=1e-12, atol=1e-12)
            np.testing.assert_allclose(bst.batch[:, a:b].cpu().numpy(), st.batch.cpu().numpy(), rtol=1e-12,
                                       atol=1e-12)
    finally:
        ctx.set_tiles(0)


def test_tiled_batch_beyond_residency_refused_cleanly(ctx):
    """A tiled batch whose workgroups cannot all be resident is refused on
    the host (nothing enqueued, no stale runtime error left behind)."""
    prob = W.make_hh_problem(4096, 0.02, 410, require_spike=False)
    B = 256
    batch = P.PackedBatch.pack([prob.X0] * B, [prob.p0] * B, [prob.y] * B, [prob.I] * B, list(range(B)), "fp32")
    w = P.widths_tensor(prob.w_state, prob.w_param)
    X_before = batch.X.clone()
    ctx.set_tile(2)
    ctx.set_tiles(32)
    try:
        with pytest.raises(P._lib.PimcError) as e:
            P.pimc_run_batch(ctx, prob.model, batch, seed=1, sweep0=0, w=w, n_sweeps=2)
    finally:
        ctx.set_tile(0)
        ctx.set_tiles(0)
    assert e.value.status == P._lib.PIMC_ERR_UNSUPPORTED
    assert ctx.sync() == 0
    torch.zeros(16, device="cuda").sum().item()   # the runtime holds no error
    assert torch.equal(batch.X, X_before)


def test_batch_graph_replays_equal_direct_launches(ctx, monkeypatch):
    """The batched sweep is launched through a captured graph whose kernel
    arguments are rewritten for every call; a context with graphs switched
    off launches directly.  Consecutive calls (different sweep counters,
    counts and statistics buffers, eager work in between) give the same
    chains and statistics both ways, and a second batch layout re-captures."""
    monkeypatch.setenv("PIMC_NO_GRAPHS", "1")
    direct = P.Context(0)
    monkeypatch.delenv("PIMC_NO_GRAPHS")
    Ms = [300, 129, 64, 37]
    probs = [W.make_hh_problem(M, 0.02, 420 + i, require_spike=False) for i, M in enumerate(Ms)]
    spec = probs[0].model
    w = P.widths_tensor(probs[0].w_state, probs[0].w_param)

    def run(c, layout):
        qs = probs if layout == 0 else probs[:2]
        batch = P.PackedBatch.pack([q.X0 for q in qs], [q.p0 for q in qs], [q.y for q in qs], [q.I for q in qs],
                                   list(range(len(qs))), "fp32")
        outs = []
        for sweep0, n in ((0, 5), (5, 7), (12, 3)):
            dev = batch.X.device
            st = P.SweepStats(ptrace=torch.zeros((len(qs), n, 7), dtype=torch.float64, device=dev),
                              acc=torch.zeros((len(qs), P._lib.PIMC_NACC), dtype=torch.int64, device=dev))
            P.pimc_run_batch(c, spec, batch, seed=9, sweep0=sweep0, w=w, n_sweeps=n, stats=st)
            junk = torch.randn(1 << 14, device="cuda")
            (junk * junk).sum().item()
            assert c.sync() == 0
            outs.append((batch.X.cpu().numpy().copy(), batch.p.cpu().numpy().copy(), st.ptrace.cpu().numpy(),
                         st.acc.cpu().numpy()))
        return outs

    try:
        for layout in (0, 1, 0):
            a = run(ctx, layout)
            b = run(direct, layout)
            for (Xa, pa, ta, ca), (Xb, pb, tb, cb) in zip(a, b):
                np.testing.assert_array_equal(Xa, Xb)
                np.testing.assert_array_equal(pa, pb)
                np.testing.assert_array_equal(ta, tb)
                np.testing.assert_array_equal(ca, cb)
    finally:
        direct.close()


def test_param_update_entry_point(ctx):
    prob = _problem(256)
    X = _perturbed(prob, 6)
    p = prob.p_true.copy()
    Xo, po, od, so = _oracle_one_sweep(prob, X, p, 42, flags=OS.PARAMS)
    win = P.Window.from_arrays(X, p, prob.y, prob.I, "fp64")
    w = P.widths_tensor(prob.w_state, prob.w_param)
    dbg = P.SweepDebug.allocate(win)
    P.pimc_param_update(ctx, prob.model, win, seed=prob.seed, chain=0, sweep0=42, w=w, debug=dbg)
    assert ctx.sync() == 0
    np.testing.assert_array_equal(win.X.cpu().numpy(), X)
    np.testing.assert_allclose(dbg.pdA.cpu().numpy(), od.pdA, rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(win.p.cpu().numpy(), po, rtol=1e-14)


def test_uniform_proposal_fp64(ctx):
    prob = _problem(64, proposal="uniform")
    X = _perturbed(prob, 7)
    Xo, po, od, so = _oracle_one_sweep(prob, X, prob.p_true, 3)
    win, gd, gs = _gpu_one_sweep(ctx, prob, X, prob.p_true, 3, "fp64")
    np.testing.assert_allclose(gd.xprop.cpu().numpy(), od.xprop, rtol=1e-15, atol=1e-15)
    _check_sites(gd, od, 1e-12, lambda d: 1e-6)


def test_out_of_box_state_reported(ctx):
    prob = _problem(40)
    X = prob.X0.copy()
    X[5, 1] = 1.5   # gate outside [0, 1]
    win = P.Window.from_arrays(X, prob.p0, prob.y, prob.I, "fp64")
    w = P.widths_tensor(prob.w_state, prob.w_param)
    P.pimc_sweep(ctx, prob.model, win, seed=1, chain=0, sweep0=0, w=w, n_sweeps=3)
    assert ctx.sync() == P._lib.PIMC_ERR_BOX
    np.testing.assert_array_equal(win.X.cpu().numpy(), X)   # untouched
    assert ctx.sync() == 0                                   # flag cleared


def test_nonfinite_data_reported(ctx):
    prob = _problem(40)
    y = prob.y.copy()
    y[7] = np.nan
    win = P.Window.from_arrays(prob.X0, prob.p0, y, prob.I, "fp32")
    w = P.widths_tensor(prob.w_state, prob.w_param)
    st = P.SweepStats.allocate(win, 2, moments=False)
    P.pimc_sweep(ctx, prob.model, win, seed=1, chain=0, sweep0=0, w=w, n_sweeps=2, stats=st)
    assert ctx.sync() == P._lib.PIMC_ERR_NONFINITE
    assert st.acc.cpu().numpy()[9] >= 2


@pytest.mark.parametrize("site", [257, 7])
def test_nonfinite_site_of_any_lane_reported(ctx, site):
    """A non-finite site dA is counted whichever lane owns the site: with
    M = 1000 in FP32 (4 sites per thread, 256 threads) site 257 belongs to
    lane 0 of the second wave, site 7 to lane 1 of the first."""
    prob = _problem(1000)
    y = prob.y.copy()
    y[site] = np.nan
    win = P.Window.from_arrays(prob.X0, prob.p0, y, prob.I, "fp32")
    w = P.widths_tensor(prob.w_state, prob.w_param)
    st = P.SweepStats.allocate(win, 3, moments=False)
    ctx.set_tiles(0)
    P.pimc_sweep(ctx, prob.model, win, seed=1, chain=0, sweep0=0, w=w, n_sweeps=3, stats=st)
    assert ctx.sync() == P._lib.PIMC_ERR_NONFINITE
    assert st.acc.cpu().numpy()[9] >= 3


def test_param_only_multi_sweep_fp64_lockstep(ctx):
    """Several parameter-only sweeps in one call (one workgroup, no site
    half-sweep between the moves of consecutive sweeps) follow the oracle's
    chain: every proposal, dA and decision of the last sweep and the
    parameter trace of all of them."""
    prob = _problem(1024, mask=0x7F)
    X = _perturbed(prob, 9)
    p = prob.p_true * 1.01
    n = 12
    Xo, po = X.copy(), p.copy()
    st = OS.Stats(prob.M, 4, 7, n)
    od = OS.Debug()
    OS.run(prob.model, Xo, po, prob.y, prob.I, seed=prob.seed, chain=2, sweep0=40, n_sweeps=n,
           w_state=prob.w_state, w_param=prob.w_param, flags=OS.PARAMS, stats=st, debug=od)
    ctx.set_tiles(0)
    win = P.Window.from_arrays(X, p, prob.y, prob.I, "fp64")
    gst = P.SweepStats.allocate(win, n, moments=False)
    gd = P.SweepDebug.allocate(win)
    w = P.widths_tensor(prob.w_state, prob.w_param)
    P.pimc_sweep(ctx, prob.model, win, seed=prob.seed, chain=2, sweep0=40, w=w, n_sweeps=n,
                 flags=P._lib.PIMC_PARAMS, stats=gst, debug=gd)
    assert ctx.sync() == 0
    np.testing.assert_allclose(gd.pprop.cpu().numpy(), od.pprop, rtol=1e-14)
    np.testing.assert_allclose(gd.pdA.cpu().numpy(), od.pdA, rtol=1e-9, atol=1e-9)
    np.testing.assert_array_equal(gd.paccept.cpu().numpy().astype(bool), od.paccept)
    np.testing.assert_allclose(gst.ptrace.cpu().numpy(), st.ptrace, rtol=1e-13)
    np.testing.assert_allclose(win.p.cpu().numpy(), po, rtol=1e-13)
    np.testing.assert_array_equal(win.X.cpu().numpy(), X)


def test_oversized_window_refused_on_host(ctx):
    """A window whose LDS footprint exceeds the CU's LDS, with time tiles
    disabled, is refused before anything is enqueued; the context stays
    usable."""
    prob = _problem(16384, init="truth")
    win = P.Window.from_arrays(prob.X0, prob.p0, prob.y, prob.I, "fp64")
    w = P.widths_tensor(prob.w_state, prob.w_param)
    ctx.set_tiles(1)
    try:
        with pytest.raises(P._lib.PimcError) as e:
            P.pimc_sweep(ctx, prob.model, win, seed=1, chain=0, sweep0=0, w=w, n_sweeps=1)
    finally:
        ctx.set_tiles(0)
    assert e.value.status == P._lib.PIMC_ERR_UNSUPPORTED
    assert ctx.sync() == 0
    small = P.Window.from_arrays(prob.X0[:65], prob.p0, prob.y[:65], prob.I[:65], "fp64")
    P.pimc_sweep(ctx, prob.model, small, seed=1, chain=0, sweep0=0, w=w, n_sweeps=1)
    assert ctx.sync() == 0


def test_fp64_window_limit(ctx):
    """FP64 windows run in one spill-free workgroup: M = 1024 runs, M = 1025
    is refused on the host (nothing enqueued) for every sites-per-thread
    setting."""
    prob = _problem(1025, init="truth")
    w = P.widths_tensor(prob.w_state, prob.w_param)
    ok = P.Window.from_arrays(prob.X0[:1025], prob.p0, prob.y[:1025], prob.I[:1025], "fp64")
    P.pimc_sweep(ctx, prob.model, ok, seed=1, chain=0, sweep0=0, w=w, n_sweeps=1)
    assert ctx.sync() == 0
    big = P.Window.from_arrays(prob.X0, prob.p0, prob.y, prob.I, "fp64")
    for K in (0, 4, 8):
        ctx.set_tile(K)
        try:
            with pytest.raises(P._lib.PimcError) as e:
                P.pimc_sweep(ctx, prob.model, big, seed=1, chain=0, sweep0=0, w=w, n_sweeps=1)
        finally:
            ctx.set_tile(0)
        assert e.value.status == P._lib.PIMC_ERR_UNSUPPORTED
    assert ctx.sync() == 0


def test_long_fp64_window_refused(ctx):
    """FP64 windows longer than one workgroup are refused on the host."""
    prob = _problem(16384, init="truth")
    win = P.Window.from_arrays(prob.X0, prob.p0, prob.y, prob.I, "fp64")
    w = P.widths_tensor(prob.w_state, prob.w_param)
    for T in (0, 16):
        ctx.set_tiles(T)
        try:
            with pytest.raises(P._lib.PimcError) as e:
                P.pimc_sweep(ctx, prob.model, win, seed=1, chain=0, sweep0=0, w=w, n_sweeps=1)
        finally:
            ctx.set_tiles(0)
        assert e.value.status == P._lib.PIMC_ERR_UNSUPPORTED
    assert ctx.sync() == 0


@FP64_TILES_OFF
def test_long_fp64_window_auto_tiled_lockstep(ctx):
    """FP64 window too long for one workgroup: cut into 16 tiles of 256
    threads automatically, one sweep in lockstep with the oracle."""
    prob = _problem(16384)
    X = _perturbed(prob, 9)
    p = prob.p_true * 1.005
    Xo, po, od, so = _oracle_one_sweep(prob, X, p, 3)
    win, gd, gs = _gpu_one_sweep(ctx, prob, X, p, 3, "fp64", tiles=0)
    ties = _check_sites(gd, od, 1e-12, lambda d: 1e-6)
    m = np.isfinite(od.pdA)
    np.testing.assert_allclose(gd.pdA.cpu().numpy()[m], od.pdA[m], rtol=1e-9, atol=1e-9)
    if ties == 0:
        np.testing.assert_allclose(win.X.cpu().numpy(), Xo, rtol=1e-13, atol=1e-13)
        np.testing.assert_allclose(win.p.cpu().numpy(), po, rtol=1e-14)


def test_batch_per_window_sites_per_thread(ctx, monkeypatch):
    """A batch launched with 16 sites per thread runs each window with the
    fewest of 4, 8, 12, 16 sites per thread its workgroup holds (here
    448 threads: 4, 4, 8, 12, 16, 16).  Every window's chain and statistics
    equal its run in the batch launched with 16 sites per thread for all
    windows, and its own single-window run (X bit for bit; p within 1e-14)."""
    Ms = [300, 1500, 2500, 4500, 6100, 7000]
    probs = [W.make_hh_problem(M, 0.02, 700 + i, require_spike=False) for i, M in enumerate(Ms)]
    spec = probs[0].model
    chains = [21 + i for i in range(len(Ms))]
    w = P.widths_tensor(probs[0].w_state, probs[0].w_param)
    n = 6
    monkeypatch.setenv("PIMC_BATCH_UNIFORM_K", "1")
    c2 = P.Context(0)
    monkeypatch.delenv("PIMC_BATCH_UNIFORM_K")
    outs = []
    try:
        for c in (ctx, c2):
            c.set_tile(16)
            batch = P.PackedBatch.pack([q.X0 for q in probs], [q.p0 for q in probs], [q.y for q in probs],
                                       [q.I for q in probs], chains, "fp32")
            dev = batch.X.device
            st = P.SweepStats(sum=torch.zeros(batch.X.shape, dtype=torch.float64, device=dev),
                              xref=batch.X.clone(),
                              ptrace=torch.zeros((len(Ms), n, 7), dtype=torch.float64, device=dev),
                              acc=torch.zeros((len(Ms), P._lib.PIMC_NACC), dtype=torch.int64, device=dev), burn=2)
            print(f"batch Ms={Ms} {'per-window' if c is ctx else 'uniform'} sites per thread", flush=True)
            P.pimc_run_batch(c, spec, batch, seed=31, sweep0=5, w=w, n_sweeps=n, stats=st)
            assert c.sync() == 0
            outs.append((batch, st))
            c.set_tile(0)
        (b1, s1), (b2, s2) = outs
        np.testing.assert_array_equal(b1.X.cpu().numpy(), b2.X.cpu().numpy())
        np.testing.assert_allclose(b1.p.cpu().numpy(), b2.p.cpu().numpy(), rtol=1e-14)
        np.testing.assert_array_equal(s1.acc.cpu().numpy(), s2.acc.cpu().numpy())
        np.testing.assert_allclose(s1.sum.cpu().numpy(), s2.sum.cpu().numpy(), rtol=1e-12, atol=1e-12)
        for i, q in enumerate(probs):
            win = P.Window.from_arrays(q.X0, q.p0, q.y, q.I, "fp32")
            P.pimc_sweep(ctx, spec, win, seed=31, chain=chains[i], sweep0=5, w=w, n_sweeps=n)
            assert ctx.sync() == 0
            a, b = int(b1.offsets[i]), int(b1.offsets[i + 1])
            np.testing.assert_array_equal(b1.X[a:b].cpu().numpy(), win.X.cpu().numpy())
            np.testing.assert_allclose(b1.p[i].cpu().numpy(), win.p.cpu().numpy(), rtol=1e-14)
    finally:
        c2.close()
