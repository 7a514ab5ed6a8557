"""The paper-like run (annealed initialization phase, sampling every N_skip
sweeps, the model checks of Section 6) on a shortened schedule of the
Section 5.1 window (M = 8000, dt = 0.04 ms, Ro = 100, Lorenz-driven data):
every stage runs in the library, the summary is finite and self-consistent
(beta reached 1, the steps moved, the observation errors' mean square is
about 1/Ro, the parameters stay in their box).  Statistical agreement with the
truth is the long run's business (bench.py --config paper); this checks
that the pipeline holds together."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1103_4887_amd")

pytestmark = pytest.mark.gpu


def test_paper_like_run_short():
    from paper_1103_4887_amd import replicate
    from workloads.paper_data import make_paper_problem

    prob = make_paper_problem()
    ctx = P.Context(0)
    try:
        print("paper-like run: 30000 sweeps", flush=True)
        out = replicate.run(ctx, prob, sweeps=30000, n_init=20000, n_cool=5000, n_skip=100, beta0=0.01,
                            alpha=0.02, forecast_steps=500, ensemble=64)
    finally:
        ctx.close()
    assert out["init_phase"]["beta_end"] == 1.0
    assert out["init_phase"]["site_step_factor"]["max"] > 1.05
    assert out["samples"] == 100
    pm = np.asarray(out["params"]["mean"])
    assert np.isfinite(pm).all()
    assert ((pm >= prob.model.p_lo) & (pm <= prob.model.p_hi)).all()
    e = out["errors"]
    assert np.isfinite(e["eps_msq_times_Rd"]).all()
    assert 0.3 < e["delta_msq_times_Ro"] < 3.0, e
    f = out["forecast"]
    assert np.isfinite(f["mean_state_rms_V_vs_truth"]) and 0.0 <= f["ensemble_band_5_95_covers_y"] <= 1.0
