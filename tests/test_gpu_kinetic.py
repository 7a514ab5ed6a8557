"""Moves of the Table 1 kinetic constants (PIMC_KINETIC) and windows with
their own constants, against the oracle (sampler.kinetic_moves,
action.delta_kinetic).

* action and gradient of a window whose constants differ from the model's
  equal the oracle's with those constants;
* FP64: whole sweeps (sites, parameters, the twelve constants) in lockstep:
  constants within 1e-10, every move's dA within 1e-9, decisions and
  counters equal, path within 1e-9;
* FP32 at the benchmark window's tiled shapes: each move's FP64 dA (summed
  over all tiles) equals the oracle's direct sum on the GPU's own path to
  1e-9, decisions equal where the margin exceeds 1e-6, and time tiles give
  the same chain as one workgroup.
"""

import numpy as np
import pytest

import workloads as W
from oracle import action as OA
from oracle import sampler as OS

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1103_4887_amd")

pytestmark = pytest.mark.gpu

KIN = P._lib.PIMC_KINETIC


@pytest.fixture(scope="module")
def ctx():
    c = P.Context(0)
    yield c
    c.close()


def _kin0(spec, scale=1.0):
    return np.array(spec.gates, dtype=np.float64).ravel() * scale


def _w23(prob, kin):
    return P.widths_tensor(list(prob.w_state) + list(prob.w_param), list(2e-3 * np.abs(kin)))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_action_and_grad_with_window_constants(ctx, prec):
    spec = W.ModelSpec()
    prob = W.make_hh_problem(300, 0.02, 161, model=spec, require_spike=False)
    kin = _kin0(spec) * (1.0 + 0.03 * np.sin(np.arange(12)))
    X = prob.X0.astype(np.float32).astype(np.float64)
    win = P.Window.from_arrays(X, prob.p0, prob.y, prob.I, prec)
    win.kin = torch.tensor(kin, dtype=torch.float64, device="cuda")
    spec_k = spec.with_(gates=tuple(tuple(g) for g in kin.reshape(3, 4)))
    y = prob.y.astype(np.float32).astype(np.float64) if prec == "fp32" else prob.y
    I = prob.I.astype(np.float32).astype(np.float64) if prec == "fp32" else prob.I
    out = P.pimc_action(ctx, spec, win).cpu().numpy()
    ref = OA.action(spec_k, X, y, I, prob.p0)
    np.testing.assert_allclose(out, ref, rtol=1e-12)
    if prec == "fp64":
        gX, gp = P.pimc_grad(ctx, spec, win)
        g_ref, gp_ref = OA.grad(spec_k, X, y, I, prob.p0)
        np.testing.assert_allclose(gX.cpu().numpy(), g_ref, rtol=1e-10, atol=1e-10 * np.abs(g_ref).max())
        np.testing.assert_allclose(gp.cpu().numpy(), gp_ref, rtol=1e-9)


@pytest.mark.parametrize("M,mask", [(200, 0xFFF), (97, 0x0F1)])
def test_kinetic_fp64_lockstep(ctx, M, mask):
    spec = W.ModelSpec(k_mask=mask)
    prob = W.make_hh_problem(M, 0.02, 171 + M, model=spec, require_spike=False, init="truth")
    kin0 = _kin0(spec, 1.02)
    X, p, kin = prob.X_true.copy(), np.asarray(prob.p_true, dtype=np.float64) * 1.01, kin0.copy()
    w_kin = 2e-3 * np.abs(kin0)
    n = 8
    st = OS.Stats(prob.M, 4, 7, n)
    od = OS.Debug()
    flags = OS.STATES | OS.PARAMS | OS.KINETIC
    OS.run(spec, X, p, prob.y, prob.I, seed=prob.seed, chain=2, sweep0=30, n_sweeps=n, w_state=prob.w_state,
           w_param=prob.w_param, flags=flags, stats=st, debug=od, kin=kin, w_kin=w_kin)
    ctx.set_tiles(0)
    win = P.Window.from_arrays(prob.X_true, np.asarray(prob.p_true) * 1.01, prob.y, prob.I, "fp64")
    win.kin = torch.tensor(kin0, dtype=torch.float64, device="cuda")
    gst = P.SweepStats.allocate(win, n, moments=False)
    gst.kacc = torch.zeros(12, dtype=torch.int64, device="cuda")
    gd = P.SweepDebug.allocate(win, sites=False, kinetic=True)
    print(f"kinetic fp64 lockstep M={M} mask={mask:#x}", flush=True)
    P.pimc_sweep(ctx, spec, win, seed=prob.seed, chain=2, sweep0=30, w=_w23(prob, kin0), n_sweeps=n,
                 flags=P._lib.PIMC_STATES | P._lib.PIMC_PARAMS | KIN, stats=gst, debug=gd)
    assert ctx.sync() == 0
    on = np.array([(mask >> i) & 1 for i in range(12)], dtype=bool)
    np.testing.assert_allclose(gd.kprop.cpu().numpy()[on], od.kprop[on], rtol=1e-14)
    np.testing.assert_allclose(gd.kdA.cpu().numpy()[on], od.kdA[on], rtol=1e-9, atol=1e-9)
    np.testing.assert_array_equal(gd.kaccept.cpu().numpy().astype(bool)[on], od.kaccept[on])
    np.testing.assert_allclose(win.kin.cpu().numpy(), kin, rtol=1e-10)
    np.testing.assert_array_equal(gst.acc.cpu().numpy(), st.acc)
    np.testing.assert_array_equal(gst.kacc.cpu().numpy(), st.kacc)
    np.testing.assert_allclose(win.X.cpu().numpy(), X, rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(win.p.cpu().numpy(), p, rtol=1e-10)
    assert st.kacc[on].sum() > 0          # some constants moved


@pytest.mark.parametrize("K,T", [(2, 16), (0, 0), (0, 4)])
def test_kinetic_fp32_moves_match_direct_sum(ctx, K, T):
    spec = W.ModelSpec(k_mask=0xFFF)
    prob = W.make_hh_problem(4096, 0.02, 102, model=spec, init="truth")
    kin0 = _kin0(spec, 0.99)
    ctx.set_tile(K)
    ctx.set_tiles(T)
    try:
        win = P.Window.from_arrays(prob.X_true, prob.p_true, prob.y, prob.I, "fp32")
        win.kin = torch.tensor(kin0, dtype=torch.float64, device="cuda")
        gd = P.SweepDebug.allocate(win, sites=False, kinetic=True)
        print(f"kinetic fp32 M=4096 K={K} T={T}", flush=True)
        P.pimc_sweep(ctx, spec, win, seed=prob.seed, chain=0, sweep0=12, w=_w23(prob, kin0), n_sweeps=1,
                     flags=P._lib.PIMC_STATES | P._lib.PIMC_PARAMS | KIN, debug=gd)
        assert ctx.sync() == 0
    finally:
        ctx.set_tile(0)
        ctx.set_tiles(0)
    Xg = win.X.cpu().numpy().astype(np.float64)
    pg = win.p.cpu().numpy()
    I32 = prob.I.astype(np.float32).astype(np.float64)
    kprop = gd.kprop.cpu().numpy()
    kdA = gd.kdA.cpu().numpy()
    kacc = gd.kaccept.cpu().numpy().astype(bool)
    from oracle import philox as ph
    cur = kin0.copy()
    for i in range(12):
        prop = cur.copy()
        prop[i] = kprop[i]
        s0 = spec.with_(gates=tuple(tuple(g) for g in cur.reshape(3, 4)))
        ref = OA.delta_kinetic(s0, Xg, I32, pg, prop.reshape(3, 4))
        assert kdA[i] == pytest.approx(ref, rel=1e-9, abs=1e-9), i
        u = float(ph.uniform_open(ph.draw(prob.seed, 0, i, 12, ph.TAG_KIN)[0, 2]))
        if abs(ref + np.log(u)) > 1e-6:
            assert kacc[i] == (np.log(u) < -ref), i
        if kacc[i]:
            cur = prop
    np.testing.assert_allclose(win.kin.cpu().numpy(), cur, rtol=1e-15)


def test_kinetic_fp32_tiles_give_the_same_chain(ctx):
    spec = W.ModelSpec(k_mask=0xFFF)
    prob = W.make_hh_problem(4096, 0.02, 102, model=spec, init="truth")
    kin0 = _kin0(spec, 1.01)
    outs = []
    for K, T in ((0, 0), (2, 16), (0, 8)):
        ctx.set_tile(K)
        ctx.set_tiles(T)
        try:
            win = P.Window.from_arrays(prob.X_true, prob.p_true, prob.y, prob.I, "fp32")
            win.kin = torch.tensor(kin0, dtype=torch.float64, device="cuda")
            st = P.SweepStats.allocate(win, 10, moments=False)
            P.pimc_sweep(ctx, spec, win, seed=3, chain=1, sweep0=0, w=_w23(prob, kin0), n_sweeps=10,
                         flags=P._lib.PIMC_STATES | P._lib.PIMC_PARAMS | KIN, stats=st)
            assert ctx.sync() == 0
        finally:
            ctx.set_tile(0)
            ctx.set_tiles(0)
        outs.append((win.X.cpu().numpy(), win.p.cpu().numpy(), win.kin.cpu().numpy(), st.acc.cpu().numpy()))
    for o in outs[1:]:
        np.testing.assert_array_equal(o[0], outs[0][0])
        np.testing.assert_allclose(o[1], outs[0][1], rtol=1e-14)
        np.testing.assert_allclose(o[2], outs[0][2], rtol=1e-14)
        np.testing.assert_array_equal(o[3], outs[0][3])


def test_kinetic_needs_window_constants_and_no_batch(ctx):
    spec = W.ModelSpec(k_mask=0x3)
    prob = W.make_hh_problem(64, 0.02, 101, model=spec, require_spike=False)
    win = P.Window.from_arrays(prob.X0, prob.p0, prob.y, prob.I, "fp64")
    w = _w23(prob, _kin0(spec))
    with pytest.raises(P._lib.PimcError) as e:
        P.pimc_sweep(ctx, spec, win, seed=1, chain=0, sweep0=0, w=w, n_sweeps=1,
                     flags=P._lib.PIMC_STATES | KIN)
    assert e.value.status == P._lib.PIMC_ERR_ARG
    b = P.PackedBatch.pack([prob.X0], [prob.p0], [prob.y], [prob.I], [0], "fp64")
    with pytest.raises(P._lib.PimcError) as e:
        P.pimc_run_batch(ctx, spec, b, seed=1, sweep0=0, w=w, n_sweeps=1, flags=P._lib.PIMC_STATES | KIN)
    assert e.value.status == P._lib.PIMC_ERR_ARG
    assert ctx.sync() == 0
