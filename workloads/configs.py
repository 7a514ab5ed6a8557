"""The five synthetic HH workloads (sizes, precisions, sweep counts, seeds).

c1  plain Metropolis, FP64, M=256, dt=0.02 ms, p2/p4/p6 sampled, 2000 sweeps
c2  M=4096, FP32 sites + FP64 reductions, all 7 parameters, 1e5 sweeps
c3  M=65536, dt=0.01 ms, FP32/FP64, all 7 parameters, 2e4 sweeps
c4  512 windows, M uniform in [512, 8192], per-window data and true
    parameters within +-20% of the c1 values, 1e4 sweeps
c5  HMC, M=16384, 64 chains on one dataset, 20 leapfrog steps
"""

from __future__ import annotations

import numpy as np

from .hh_data import make_hh_problem
from .problem import P_STAR, ModelSpec

# mask bits: bit l <=> p_{l+1}; c1 samples the three conductances g_Na, g_K, g_L
MASK_C1 = (1 << 1) | (1 << 3) | (1 << 5)
MASK_ALL = 0x7F

CONFIGS = {
    "c1": dict(M=256, dt=0.02, prec="fp64", p_mask=MASK_C1, sweeps=2000, burn=1000,
               chains=1, data_seed=101),
    "c2": dict(M=4096, dt=0.02, prec="fp32", p_mask=MASK_ALL, sweeps=100000, burn=50000,
               chains=1, data_seed=102),
    "c3": dict(M=65536, dt=0.01, prec="fp32", p_mask=MASK_ALL, sweeps=20000, burn=10000,
               chains=1, data_seed=103),
    "c4": dict(B=512, M_lo=512, M_hi=8192, dt=0.02, prec="fp32", p_mask=MASK_ALL,
               sweeps=10000, burn=5000, data_seed=104),
    "c5": dict(M=16384, dt=0.02, prec="fp32", p_mask=MASK_ALL, chains=64, leapfrog=20,
               warmup=1000, proposals=4000, data_seed=105),
}


def config_problem(name: str, **kw):
    """Problem for a single-window config (c1, c2, c3, c5)."""
    c = CONFIGS[name]
    model = ModelSpec(dt=c["dt"], p_mask=c["p_mask"])
    return make_hh_problem(c["M"], c["dt"], c["data_seed"], model=model, **kw)


def batch_sizes(B: int = 512, M_lo: int = 512, M_hi: int = 8192, seed: int = 104) -> np.ndarray:
    """Uneven window lengths of the batched workload, uniform in [M_lo, M_hi]."""
    rng = np.random.default_rng(seed)
    return rng.integers(M_lo, M_hi + 1, size=B)


def batch_true_params(B: int, seed: int = 104) -> np.ndarray:
    """Per-window true parameters: the Table 2 values scaled by U(0.8, 1.2)."""
    rng = np.random.default_rng(seed + 1)
    return np.asarray(P_STAR) * rng.uniform(0.8, 1.2, size=(B, 7))


def _batch_window(args):
    w, M, p_true, dt, mask, data_seed = args
    model = ModelSpec(dt=dt, p_mask=mask)
    return make_hh_problem(int(M), dt, data_seed + w, model=model, p_true=p_true, chain=w, require_spike=False)


def config_batch(name: str = "c4", B: int | None = None, workers: int = 8):
    """The windows of the batched workload: own sizes, drives, noise and true parameters."""
    c = CONFIGS[name]
    B = B or c["B"]
    sizes = batch_sizes(c["B"], c["M_lo"], c["M_hi"], c["data_seed"])[:B]
    ptrue = batch_true_params(c["B"], c["data_seed"])[:B]
    jobs = [(w, sizes[w], ptrue[w], c["dt"], c["p_mask"], c["data_seed"]) for w in range(B)]
    if workers <= 1:
        return [_batch_window(j) for j in jobs]
    import multiprocessing as mp
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(_batch_window, jobs, chunksize=4)
