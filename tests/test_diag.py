"""ESS / MCSE estimators against the closed form of an AR(1) chain.

For x_t = phi x_{t-1} + e_t the integrated autocorrelation time is
(1 + phi) / (1 - phi), so ESS = n (1 - phi) / (1 + phi)."""

import numpy as np
import pytest

from paper_1103_4887_amd import diag


@pytest.mark.parametrize("phi", [0.0, 0.5, 0.9])
def test_ess_ar1(phi):
    rng = np.random.default_rng(1)
    n = 200000
    e = rng.standard_normal(n)
    x = np.empty(n)
    x[0] = e[0] / np.sqrt(1 - phi * phi)
    for t in range(1, n):
        x[t] = phi * x[t - 1] + e[t]
    expect = n * (1 - phi) / (1 + phi)
    assert diag.ess(x) == pytest.approx(expect, rel=0.1)


def test_ess_constant_and_short():
    assert diag.ess(np.ones(100)) == 0.0
    assert diag.ess(np.arange(3.0)) == 3.0


def test_batch_mcse_matches_iid_error():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((64000, 3))
    se = diag.batch_mcse(x, nb=32)
    assert np.allclose(se, 1 / np.sqrt(64000), rtol=0.35)
