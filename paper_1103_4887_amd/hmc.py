"""HMC driver: pilot masses, step-size tuning, sampling.

* inverse masses: per state component the posterior variance averaged over
  sites, per parameter its variance, from a short pilot run of the
  Metropolis sweep on the same windows (a diagonal mass matrix);
* step size: dual averaging towards a target acceptance during warm-up
  (Hoffman & Gelman, JMLR 2014, Algorithm 5), then frozen;
* sampling: one library call that replays the captured proposal graph.
Every proposal runs in the library's kernels; this module only schedules.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L
from .api import Context, HmcStats, PackedBatch, SweepStats, pimc_hmc, pimc_run_batch


@dataclass
class HmcTuning:
    eps: float
    minv: np.ndarray
    warmup_accept: float


def pilot_minv(ctx: Context, spec, batch: PackedBatch, w: torch.Tensor, *, seed: int, sweeps: int = 2000,
               floor: float = 1e-12) -> np.ndarray:
    """Inverse masses from a pilot run of the Metropolis sweep (second half)."""
    B = batch.B
    dev = batch.X.device
    pil = PackedBatch(offsets=batch.offsets, X=batch.X.clone(), p=batch.p.clone(), y=batch.y, I=batch.I,
                      chain=batch.chain, prec=batch.prec)
    st = SweepStats(sum=torch.zeros(batch.X.shape, dtype=torch.float64, device=dev),
                    sumsq=torch.zeros(batch.X.shape, dtype=torch.float64, device=dev),
                    xref=pil.X.clone(), ptrace=torch.zeros((B, sweeps, 7), dtype=torch.float64, device=dev),
                    acc=torch.zeros((B, L.PIMC_NACC), dtype=torch.int64, device=dev), burn=sweeps // 2, stride=1)
    pimc_run_batch(ctx, spec, pil, seed=seed, sweep0=0, w=w, n_sweeps=sweeps, stats=st)
    if ctx.sync() != 0:
        raise RuntimeError("pilot run reported a device error")
    n = sweeps - sweeps // 2
    mean = st.sum.cpu().numpy() / n
    var = st.sumsq.cpu().numpy() / n - mean * mean
    minv = np.empty(11)
    minv[:4] = np.maximum(var.mean(axis=0), floor)
    tr = st.ptrace.cpu().numpy()[:, sweeps // 2:, :]
    minv[4:] = np.maximum(tr.var(axis=1).mean(axis=0), floor)
    return minv


def tune_eps(ctx: Context, spec, batch: PackedBatch, minv: np.ndarray, *, seed: int, L_steps: int,
             warmup: int, eps0: float, target: float = 0.7, k0: int = 0) -> HmcTuning:
    """Dual-averaging step size over `warmup` proposals (k0 .. k0+warmup-1)."""
    mu = math.log(10.0 * eps0)
    gamma, t0, kappa = 0.05, 10.0, 0.75
    Hbar, log_eps_bar = 0.0, 0.0
    eps = eps0
    acc_hist = []
    for m in range(1, warmup + 1):
        st = HmcStats.allocate(batch.B, 1, device=batch.X.device)
        pimc_hmc(ctx, spec, batch, seed=seed, k0=k0 + m - 1, eps=eps, L_steps=L_steps, minv=minv, n_proposals=1,
                 stats=st)
        if ctx.sync() != 0:
            raise RuntimeError("warm-up proposal reported a device error")
        dH = st.dH.cpu().numpy()[:, 0]
        left = st.acc.cpu().numpy()[:, 1] > 0
        a = np.where(np.isfinite(dH) & ~left, np.minimum(1.0, np.exp(-np.nan_to_num(dH, nan=np.inf))), 0.0)
        am = float(a.mean())
        acc_hist.append(am)
        Hbar = (1 - 1 / (m + t0)) * Hbar + (target - am) / (m + t0)
        log_eps = mu - math.sqrt(m) / gamma * Hbar
        eta = m ** (-kappa)
        log_eps_bar = eta * log_eps + (1 - eta) * log_eps_bar
        eps = math.exp(log_eps)
    return HmcTuning(eps=math.exp(log_eps_bar), minv=minv, warmup_accept=float(np.mean(acc_hist[-50:])))


def sample(ctx: Context, spec, batch: PackedBatch, tuning: HmcTuning, *, seed: int, L_steps: int, n: int,
           k0: int) -> HmcStats:
    st = HmcStats.allocate(batch.B, n, device=batch.X.device)
    pimc_hmc(ctx, spec, batch, seed=seed, k0=k0, eps=tuning.eps, L_steps=L_steps, minv=tuning.minv, n_proposals=n,
             stats=st)
    if ctx.sync() != 0:
        raise RuntimeError("HMC sampling reported a device error")
    return st
