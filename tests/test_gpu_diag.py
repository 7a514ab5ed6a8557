"""Model checks (pimc_model_errors, pimc_forecast) against the oracle
(oracle/diagnostics.py): per-link model and observation errors summed over
two calls within 1e-12 (their squares through the roots, within 1e-13 of
the largest component), forecasts (deterministic and with model noise) of a
small ensemble within 1e-10 (FP64 both sides; the noise uses the same Philox
normals)."""

import numpy as np
import pytest

import workloads as W
from oracle import diagnostics as OD

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1103_4887_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = P.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_model_errors_match_oracle(ctx, prec):
    prob = W.make_hh_problem(700, 0.02, 191, require_spike=False)
    X = prob.X0.astype(np.float32).astype(np.float64)
    win = P.Window.from_arrays(X, prob.p0, prob.y, prob.I, prec)
    esum = torch.zeros((prob.M, 5), dtype=torch.float64, device="cuda")
    esq = torch.zeros_like(esum)
    for _ in range(2):
        P.pimc_model_errors(ctx, prob.model, win, esum, esq)
    torch.cuda.synchronize()
    y = prob.y if prec == "fp64" else prob.y.astype(np.float32).astype(np.float64)
    I = prob.I if prec == "fp64" else prob.I.astype(np.float32).astype(np.float64)
    e, d = OD.model_errors(prob.model, X, y, I, prob.p0)
    ref = np.concatenate([e, d[:, None]], axis=1)
    np.testing.assert_allclose(esum.cpu().numpy(), 2 * ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    # the squares through their roots: an error term is a difference of O(x)
    # quantities, so its own rounding is absolute (about 1e-13 of the
    # component's scale), which the square turns into a relative error
    # where the term is tiny
    scale = np.concatenate([np.abs(X).max(axis=0), [np.abs(y).max()]])
    np.testing.assert_allclose(np.sqrt(esq.cpu().numpy() / 2), np.abs(ref), rtol=1e-11, atol=1e-13 * scale.max())


@pytest.mark.parametrize("noise", [0.0, 1.0])
def test_forecast_matches_oracle(ctx, noise):
    prob = W.make_hh_problem(200, 0.02, 193, require_spike=False, init="truth")
    spec = prob.model
    B, N = 5, 400
    rng = np.random.default_rng(2)
    x0 = prob.X_true[-B:] + 0.0
    p = np.asarray(prob.p_true)[None, :] * (1.0 + 0.01 * rng.standard_normal((B, 7)))
    I = 6.0 + 3.0 * np.sin(np.arange(N + 1) * 0.05)
    out = P.pimc_forecast(ctx, spec, torch.tensor(x0, device="cuda"), torch.tensor(p, device="cuda"),
                          torch.tensor(I, device="cuda"), N, noise=noise, seed=77, member0=10)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for b in range(B):
        ref = OD.forecast(spec, x0[b], p[b], I, N, noise=noise, seed=77, member=10 + b)
        np.testing.assert_allclose(got[b], ref, rtol=1e-10, atol=1e-10)
