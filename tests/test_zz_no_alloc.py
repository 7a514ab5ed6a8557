"""The allocation-free action (pimc_action_noalloc) against pimc_action.

Two calls in a row on the same GPU, the second on a smaller window (the
library's fixed workspace keeps the first call's partials; the second must
not see them), then the largest window the workspace holds and one beyond,
which is refused before anything runs.  Bars: equal to pimc_action bit for
bit (same kernels, same reduction order), and within 1e-12 of the oracle.
"""

import numpy as np
import pytest

import workloads as W
from oracle import action as OA

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1103_4887_amd")

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_action_equals_action(prec):
    ctx = P.Context(0)
    try:
        for M, seed in ((5000, 181), (300, 182)):
            prob = W.make_hh_problem(M, 0.02, seed, require_spike=False)
            win = P.Window.from_arrays(prob.X0, prob.p0, prob.y, prob.I, prec)
            ref = P.pimc_action(ctx, prob.model, win).cpu().numpy()
            out = torch.full((3,), float("nan"), dtype=torch.float64, device="cuda")
            print(f"noalloc action {prec} M={M}", flush=True)
            P.pimc_action_noalloc(prob.model, win, out)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(out.cpu().numpy(), ref)
            X = prob.X0 if prec == "fp64" else prob.X0.astype(np.float32).astype(np.float64)
            y = prob.y if prec == "fp64" else prob.y.astype(np.float32).astype(np.float64)
            I = prob.I if prec == "fp64" else prob.I.astype(np.float32).astype(np.float64)
            np.testing.assert_allclose(out.cpu().numpy(), OA.action(prob.model, X, y, I, prob.p0), rtol=1e-12)
    finally:
        ctx.close()


def test_noalloc_action_size_limit():
    lim = P._lib.PIMC_NOALLOC_MAX_SITES
    spec = W.ModelSpec()
    for M, ok in ((lim - 1, True), (lim, False)):
        X = torch.zeros((M + 1, 4), dtype=torch.float32, device="cuda")
        X[:, 0] = -65.0
        X[:, 1:] = 0.3
        win = P.Window(X=X, p=torch.tensor(W.P_STAR, dtype=torch.float64, device="cuda"),
                       y=torch.full((M + 1,), -65.0, dtype=torch.float32, device="cuda"),
                       I=torch.zeros(M + 1, dtype=torch.float32, device="cuda"), prec="fp32")
        out = torch.full((3,), float("nan"), dtype=torch.float64, device="cuda")
        if ok:
            P.pimc_action_noalloc(spec, win, out)
            torch.cuda.synchronize()
            ctx = P.Context(0)
            try:
                np.testing.assert_array_equal(out.cpu().numpy(), P.pimc_action(ctx, spec, win).cpu().numpy())
            finally:
                ctx.close()
        else:
            with pytest.raises(P._lib.PimcError) as e:
                P.pimc_action_noalloc(spec, win, out)
            assert e.value.status == P._lib.PIMC_ERR_UNSUPPORTED
            assert torch.isnan(out).all()
