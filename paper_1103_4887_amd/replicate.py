"""The paper-like run of Section 5.1 and the model checks of Section 6.

Schedules library calls only (every sweep, error sum and forecast runs in
the library's kernels; tensors move to the host only for the summary):

1. initialization phase (Section 4.2): N_init sweeps with simulated
   annealing of beta from beta0 over N_cool sweeps and the step-size rule
   every N_skip sweeps (pimc_sweep_init);
2. sampling: the remaining sweeps in calls of N_skip sweeps (the adjusted
   steps stay in use, beta = 1); after the last sweep of every call (every
   N_skip-th path update, Section 4.1) the path moments, the parameters, the
   model and observation errors of the path (pimc_model_errors) and the
   final state x_M are taken (x_M and p for the ensemble forecast);
3. summary: parameter means and standard deviations against the truth
   (Table 2), the share of unobserved path components whose truth lies
   within 4 standard deviations of the mean (the band of Fig. 4), the error
   statistics of Section 6 (<eps_n>, <delta_n>, their variances against
   1/Rd and 1/Ro, where <eps_V> departs from zero relative to the spikes),
   a forecast from <x_M>, <p> and a noisy ensemble forecast from the last
   posterior samples, compared with the continuation of the data.
"""

from __future__ import annotations

import time
from typing import Optional

import numpy as np
import torch

from . import _lib as L
from . import autotune
from .api import (Context, InitPhase, SweepStats, Window, pimc_forecast, pimc_model_errors, pimc_sweep_init,
                  widths_tensor)


def run(ctx: Context, prob, *, sweeps: int, n_init: int, n_cool: int, n_skip: int, beta0: float = 0.01,
        f_acc: float = 0.23, alpha: float = 0.02, prec: str = "fp32", forecast_steps: int = 1000,
        ensemble: int = 256, seed: Optional[int] = None, verbose: bool = False) -> dict:
    spec = prob.model
    seed = prob.seed if seed is None else seed
    dev = "cuda"
    win = Window.from_arrays(prob.X0, prob.p0, prob.y, prob.I, prec)
    w = widths_tensor(prob.w_state, prob.w_param)
    shape = autotune.tune(ctx, spec, win, w, narrow=True)
    # the tuner ran on a scratch copy; start from the initial guess
    ip = InitPhase.start(win, prob.w_param, beta0=beta0, n_cool=n_cool, n_init=n_init, n_skip=n_skip,
                         f_acc=f_acc, alpha=alpha)
    t0 = time.perf_counter()
    tr_init = SweepStats(ptrace=torch.zeros((n_init, 7), dtype=torch.float64, device=dev),
                         acc=torch.zeros(L.PIMC_NACC, dtype=torch.int64, device=dev))
    if n_init > 0:
        pimc_sweep_init(ctx, spec, win, seed=seed, chain=0, sweep0=0, w=w, n_sweeps=n_init, init=ip, stats=tr_init)
        if ctx.sync() != 0:
            raise RuntimeError("device error in the initialization phase")
    t_init = time.perf_counter() - t0
    if verbose:
        print(f"initialization phase: {n_init} sweeps in {t_init:.1f} s", flush=True)
    M = prob.M
    n_samp = (sweeps - n_init) // n_skip
    st = SweepStats(sum=torch.zeros((M + 1, 4), dtype=torch.float64, device=dev),
                    sumsq=torch.zeros((M + 1, 4), dtype=torch.float64, device=dev), xref=win.X.clone(),
                    acc=torch.zeros(L.PIMC_NACC, dtype=torch.int64, device=dev), burn=n_init + n_skip - 1,
                    stride=n_skip)
    esum = torch.zeros((M, 5), dtype=torch.float64, device=dev)
    esq = torch.zeros_like(esum)
    ptr = torch.zeros((n_samp, n_skip, 7), dtype=torch.float64, device=dev)
    xM = torch.zeros((n_samp, 4), dtype=torch.float64, device=dev)
    pS = torch.zeros((n_samp, 7), dtype=torch.float64, device=dev)
    t1 = time.perf_counter()
    for i in range(n_samp):
        k0 = n_init + i * n_skip
        st.ptrace = ptr[i]
        pimc_sweep_init(ctx, spec, win, seed=seed, chain=0, sweep0=k0, w=w, n_sweeps=n_skip, init=ip, stats=st)
        pimc_model_errors(ctx, spec, win, esum, esq)
        xM[i] = win.X[M].to(torch.float64)
        pS[i] = win.p
    if ctx.sync() != 0:
        raise RuntimeError("device error in the sampling phase")
    t_samp = time.perf_counter() - t1
    if verbose:
        print(f"sampling: {n_samp * n_skip} sweeps, {n_samp} samples in {t_samp:.1f} s", flush=True)

    # ---- summary ----------------------------------------------------------
    out = {"M": M, "dt": spec.dt, "Ro": spec.Ro, "sweeps": sweeps, "n_init": n_init, "n_cool": n_cool,
           "n_skip": n_skip, "beta0": beta0, "f_acc": f_acc, "alpha": alpha, "prec": prec,
           "launch": {"K": shape[0], "tiles": shape[1]}, "samples": n_samp,
           "wall_s": {"init": t_init, "sampling": t_samp},
           "us_per_sweep": 1e6 * (t_init + t_samp) / max(1, sweeps)}
    beta_end = float(ip.beta.cpu().numpy()[0])
    scale = ip.site_scale.cpu().numpy()
    out["init_phase"] = {"beta_end": beta_end, "site_step_factor": {"min": float(scale.min()),
                                                                    "median": float(np.median(scale)),
                                                                    "max": float(scale.max())},
                         "param_steps": [float(v) for v in ip.w_param.cpu().numpy()]}
    # parameters from the sampled trace (one value per N_skip sweeps, Section 4.1)
    pt = ptr[:, -1, :].cpu().numpy()
    pm, psd = pt.mean(axis=0), pt.std(axis=0, ddof=1)
    truth = np.asarray(prob.p_true)
    out["params"] = {"mean": pm.tolist(), "sd": psd.tolist(), "truth": truth.tolist(),
                     "z": ((pm - truth) / np.maximum(psd, 1e-300)).tolist()}
    # path: means and sds of the unobserved states, coverage of the truth by +-4 sd
    ns = n_samp
    ref = st.xref.cpu().numpy().astype(np.float64)
    mean = ref + st.sum.cpu().numpy() / ns
    var = np.maximum(st.sumsq.cpu().numpy() / ns - (st.sum.cpu().numpy() / ns) ** 2, 0.0)
    sd = np.sqrt(var)
    Xt = prob.X_true
    cover = (np.abs(Xt - mean) <= 4.0 * sd + 1e-12)
    out["path"] = {"coverage_4sd": {c: float(cover[:, j].mean()) for j, c in enumerate("Vmhn")},
                   "rms_error": {c: float(np.sqrt(((Xt[:, j] - mean[:, j]) ** 2).mean())) for j, c in enumerate("Vmhn")},
                   "median_sd": {c: float(np.median(sd[:, j])) for j, c in enumerate("Vmhn")}}
    # model and observation errors (Section 6)
    es, eq = esum.cpu().numpy() / ns, esq.cpu().numpy() / ns
    ev = np.maximum(eq - es * es, 0.0)
    Rd = np.asarray(spec.Rd, dtype=np.float64)
    spikes = np.where((Xt[1:, 0] > 50.0) & (Xt[:-1, 0] <= 50.0))[0] + 1
    top = np.argsort(-np.abs(es[:, 0]))[:max(1, M // 100)] + 1     # links with the largest |<eps_V>|
    near = np.array([np.min(np.abs(spikes - n)) <= int(round(1.0 / spec.dt)) if len(spikes) else False
                     for n in top])
    # Section 6: over the samples and the window, the errors should have zero
    # mean and second moments 1/Rd and 1/Ro; the per-site spread across
    # samples (the posterior uncertainty of each error) is reported beside
    out["errors"] = {
        "eps_mean_abs_avg": np.abs(es[:, :4]).mean(axis=0).tolist(),
        "eps_msq_times_Rd": (eq[:, :4].mean(axis=0) * Rd).tolist(),
        "eps_posterior_var_times_Rd": (ev[:, :4].mean(axis=0) * Rd).tolist(),
        "delta_mean": float(es[:, 4].mean()), "delta_msq_times_Ro": float(eq[:, 4].mean() * spec.Ro),
        "delta_posterior_var_times_Ro": float(ev[:, 4].mean() * spec.Ro),
        "top1pct_abs_epsV_within_1ms_of_spike": float(near.mean()), "spikes": int(len(spikes))}
    # forecasts from the end of the window over the continuation of the drive
    Ifut = np.asarray(prob.meta["I_future"], dtype=np.float64)[:forecast_steps + 1]
    N = len(Ifut) - 1
    Xfut = np.asarray(prob.meta["X_future"])[:N + 1]
    yfut = np.asarray(prob.meta["y_future"])[:N + 1]
    I_d = torch.tensor(Ifut, device=dev)
    x_mean = xM.mean(dim=0, keepdim=True)
    p_mean = pS.mean(dim=0, keepdim=True)
    det = pimc_forecast(ctx, spec, x_mean, p_mean, I_d, N)[0].cpu().numpy()
    E = min(ensemble, n_samp)
    ens = pimc_forecast(ctx, spec, xM[-E:].contiguous(), pS[-E:].contiguous(), I_d, N, noise=1.0, seed=seed + 99)
    ens = ens.cpu().numpy()
    lo, hi = np.percentile(ens[:, :, 0], 5, axis=0), np.percentile(ens[:, :, 0], 95, axis=0)
    out["forecast"] = {"steps": N, "ms": N * spec.dt,
                       "mean_state_rms_V_vs_truth": float(np.sqrt(((det[:, 0] - Xfut[:, 0]) ** 2).mean())),
                       "ensemble": E, "ensemble_band_5_95_covers_y": float(((yfut >= lo) & (yfut <= hi)).mean()),
                       "ensemble_mean_rms_V_vs_truth": float(np.sqrt(((ens[:, :, 0].mean(axis=0) - Xfut[:, 0]) ** 2).mean()))}
    acc = st.acc.cpu().numpy()
    out["accept"] = {"sites": float(acc[:2].sum() / ((M + 1) * n_samp * n_skip)),
                     "params": (acc[2:9] / (n_samp * n_skip)).tolist()}
    return out
