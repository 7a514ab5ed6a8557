"""Posterior agreement of the FP32 sampler with the FP64 oracle.

The site-parity tests tie every FP32 decision to the oracle's wherever the
margin allows.  This test checks the aggregate: independent chains of the
FP32 path (FP32 sites, FP64 sums and accept tests) and of the FP64 oracle,
started from the same state of an HH window with all seven parameters
sampled, give the same posterior means of every state component and every
parameter within Monte Carlo error.  The MCSE of each mean is the spread of
the independent chains' means / sqrt(chains), and the decision rule is the
multiple-testing rule for posterior comparisons: every parameter within 3
MCSE, at most 1 % of the state components beyond 3 and none beyond 5.

Inputs: the HH twin experiment of Section 5.1 (Table 1 gates, Table 2 true
parameters), M = 127 steps at dt = 0.02 ms, chains started at the true path
and parameters; the oracle gets the same FP32-rounded path, data and drive
as the GPU.
"""

import multiprocessing as mp
import os

import numpy as np
import pytest

import workloads as W
from oracle import sampler as OS

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1103_4887_amd")

pytestmark = pytest.mark.gpu

M, N, BURN, SEED = 127, 1600, 400, 2024
CHAINS_GPU, CHAINS_ORACLE = 64, 32


def _problem():
    prob = W.make_hh_problem(M=M, dt=0.02, init="truth", require_spike=False)
    r32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    return prob, r32(prob.X0), r32(prob.y), r32(prob.I)


def _oracle_chain(chain):
    prob, X0, y, I = _problem()
    X, p = X0.copy(), prob.p0.copy()
    st = OS.Stats(M, 4, 7, N, burn=BURN, xref=X0.copy())
    OS.run(prob.model, X, p, y, I, seed=SEED, chain=chain, sweep0=0, n_sweeps=N,
           w_state=prob.w_state, w_param=prob.w_param, stats=st)
    return X0 + st.sum / st.n_post, st.ptrace[BURN:].mean(axis=0)


def _z(a, b):
    """Two-sample z of the means of per-chain values a [Ca, ...], b [Cb, ...]."""
    se2 = a.var(axis=0, ddof=1) / len(a) + b.var(axis=0, ddof=1) / len(b)
    d = a.mean(axis=0) - b.mean(axis=0)
    assert np.all(se2 > 0), "a component did not move in any chain"
    return d / np.sqrt(se2)


def test_fp32_chains_match_oracle_posterior_means():
    prob, X0, y, I = _problem()
    assert prob.model.p_mask == 0x7F
    workers = max(1, min(16, os.cpu_count() or 1))
    print(f"oracle: {CHAINS_ORACLE} chains x {N} sweeps, M={M}, {workers} workers", flush=True)
    with mp.get_context("fork").Pool(workers) as pool:
        res = pool.map(_oracle_chain, range(CHAINS_ORACLE), chunksize=1)
    xs_o = np.stack([r[0] for r in res])
    ps_o = np.stack([r[1] for r in res])

    print(f"gpu: {CHAINS_GPU} chains x {N} sweeps (fp32 batch)", flush=True)
    ctx = P.Context(0)
    try:
        chains = list(range(1000, 1000 + CHAINS_GPU))
        batch = P.PackedBatch.pack([X0] * CHAINS_GPU, [prob.p0] * CHAINS_GPU, [y] * CHAINS_GPU,
                                   [I] * CHAINS_GPU, chains, "fp32")
        dev = batch.X.device
        st = P.SweepStats(sum=torch.zeros(batch.X.shape, dtype=torch.float64, device=dev),
                          xref=batch.X.clone(),
                          ptrace=torch.zeros((CHAINS_GPU, N, 7), dtype=torch.float64, device=dev),
                          acc=torch.zeros((CHAINS_GPU, P._lib.PIMC_NACC), dtype=torch.int64, device=dev),
                          burn=BURN)
        w = P.widths_tensor(prob.w_state, prob.w_param)
        P.pimc_run_batch(ctx, prob.model, batch, seed=SEED, sweep0=0, w=w, n_sweeps=N, stats=st)
        assert ctx.sync() == 0
        xref = st.xref.cpu().numpy().astype(np.float64)
        xs_g = (xref + st.sum.cpu().numpy() / (N - BURN)).reshape(CHAINS_GPU, M + 1, 4)
        ps_g = st.ptrace.cpu().numpy()[:, BURN:].mean(axis=1)
    finally:
        ctx.close()

    zp = _z(ps_g, ps_o)
    zx = _z(xs_g, xs_o).ravel()
    print("parameter z:", np.round(zp, 2), flush=True)
    big = np.flatnonzero(np.abs(zx) > 3.0)
    print(f"state z: max |z| {np.abs(zx).max():.2f}, beyond 3: {len(big)} of {zx.size}",
          [(int(i) // 4, "Vmhn"[int(i) % 4], round(float(zx[i]), 2)) for i in big], flush=True)
    assert np.all(np.abs(zp) <= 3.0), zp
    assert (np.abs(zx) > 3.0).sum() <= 0.01 * zx.size
    assert np.all(np.abs(zx) <= 5.0)
