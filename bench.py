"""Throughput of the red-black Metropolis sweep on one MI355X.

One step = one sweep of the whole hot path over the window: the even and
odd half-sweeps of every site, the sequential parameter moves and the path
statistics.  Default workload: the HH window with M = 4096 steps, FP32 site
arithmetic with FP64 reductions and decisions, all seven parameters sampled,
one chain (synthetic twin-experiment data).  The timed K sweeps run as one
persistent launch between two synchronisations; every input is resident in
HBM before the timed region starts.

Prints one JSON line: site-updates/s (value), the parameters' ESS/s, the
roofline of the sweep kernel and the CPU oracle timed on a bounded sample.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "path site-updates/s + param ESS/s, HMC vs plain sweep, HH M=4096, 1 GPU"

# VALU lane-slots the method needs per FP32-mode site update (the per-unit
# figure of the measurement plan): two Philox blocks (about 200 integer
# slots, the 32x32->64 products at reduced rate), four Box-Muller normals,
# F(x') with three tanh and three reciprocals, the local dA, the FP64
# decision and the parameter sufficient-statistic terms.
SLOTS_PER_SITE_UPDATE = 500
PEAK_SLOTS_PER_S = 256 * 4 * 16 * 2.4e9     # CUs x SIMDs x lanes x clock

# HBM bytes per sweep of the benchmark shape, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE runs calibrated against a plain copy (profiles/ holds the
# summary).  They belong to one version of the kernel source: when the source
# hash differs, the traffic is reported as unknown.
TRAFFIC = {"sweep_source_sha256": "b997400030c0ef7fd32ed63f2191250528a169fbf8cab0a395141e4b0bd8d668",
           "launch": (2, 16), "fetch_bytes_per_sweep": 80.3e3, "write_bytes_per_sweep": 16.6e3}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="sweeps (proposals for c5); default 100000 for one window, 2000 for c4, 300 for c5")
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--config", default="c2",
                    help="c1-c3: one window; c4: the uneven batch; c5: HMC on 64 chains; paper: the paper-like "
                         "run of Section 5.1 with the model checks of Section 6 (default c2)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="budget of each oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tile", type=int, default=0, help="sites per thread (0: autotune)")
    ap.add_argument("--tiles", type=int, default=-1, help="time tiles per window (-1: autotune)")
    ap.add_argument("--nskip", type=int, default=10, help="path moments every nskip-th sweep (N_skip)")
    ap.add_argument("--cmp-seconds", type=float, default=20.0,
                    help="wall budget of each sampler in the HMC vs plain sweep comparison (0: skip it)")
    ap.add_argument("--cmp-chains", type=int, default=64)
    ap.add_argument("--cmp-equilibrate", type=float, default=5.0,
                    help="untimed seconds of batched sweeps that equilibrate the chains before the comparison")
    ap.add_argument("--no-sub-blocks", dest="sub_blocks", action="store_false",
                    help="c2 only: skip the short batched (c4) and HMC (c5) measurements")
    return ap.parse_args()


def kernel_source_sha256() -> str:
    """sha256 over the sweep kernel's source files (sweep.hip, sweep_body.inc,
    then layout.hpp)."""
    import hashlib
    h = hashlib.sha256()
    for name in ("sweep.hip", "sweep_body.inc", "layout.hpp"):
        with open(os.path.join(ROOT, "paper_1103_4887_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic_per_launch(shape, sweeps: int):
    sha = kernel_source_sha256()
    if sha != TRAFFIC["sweep_source_sha256"] or tuple(shape[:2]) != TRAFFIC["launch"]:
        return None
    return (TRAFFIC["fetch_bytes_per_sweep"] + TRAFFIC["write_bytes_per_sweep"]) * sweeps


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores() -> int:
    """Worker processes for the N-core oracle legs: the host cores this
    process may use, at most 16 (the share of one GPU on the box)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _oracle_worker(job):
    """One host core: the oracle on its own window for `budget` seconds.
    Runs in a spawned process that never touches the GPU."""
    os.environ["OMP_NUM_THREADS"] = "1"
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    kind, prob, budget, extra = job
    from oracle import hmc as OH
    from oracle import sampler as OS

    X, p = prob.X0.copy(), prob.p0.copy()
    n, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < budget:
        if kind == "sweep":
            OS.run(prob.model, X, p, prob.y, prob.I, seed=prob.seed, chain=0, sweep0=n, n_sweeps=1,
                   w_state=prob.w_state, w_param=prob.w_param)
        else:
            eps, L, minv = extra
            X, p, _, _ = OH.hmc_proposal(prob.model, X, p, prob.y, prob.I, seed=prob.seed, chain=0, k=n, e=eps,
                                         L=L, minv_state=minv[:4], minv_param=minv[4:])
        n += 1
    wall = time.perf_counter() - t0
    units = (prob.M + 1) * n * (1 if kind == "sweep" else extra[1])
    return units, wall, n


def cpu_baseline_ncore(kind: str, probs, budget_s: float, extra=None):
    """The oracle on every host core at once (one spawned process per core,
    each on its own window or chain); rate = all units / the longest wall."""
    import multiprocessing as mp

    ncore = host_cores()
    jobs = [(kind, probs[i % len(probs)], budget_s, extra) for i in range(ncore)]
    with mp.get_context("spawn").Pool(ncore) as pool:
        res = pool.map(_oracle_worker, jobs)
    units = sum(r[0] for r in res)
    wall = max(r[1] for r in res)
    unit = "site-updates/s" if kind == "sweep" else "site-leapfrogs/s"
    what = "sweeps" if kind == "sweep" else "HMC proposals"
    return {"value": units / wall, "unit": unit, "cores": ncore, "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"{sum(r[2] for r in res)} {what} on {ncore} processes (one window or chain each, "
                      f"M from {min(q.M for q in probs)} to {max(q.M for q in probs)}), {wall:.1f} s"}


def cpu_baseline(prob, budget_s: float):
    """The CPU oracle, untouched, on the same window for a bounded number of sweeps."""
    import numpy as np
    from oracle import sampler as OS

    X = prob.X0.copy()
    p = prob.p0.copy()
    kw = dict(seed=prob.seed, chain=0, w_state=prob.w_state, w_param=prob.w_param)
    OS.run(prob.model, X, p, prob.y, prob.I, sweep0=0, n_sweeps=1, **kw)   # warm
    n = 0
    t0 = time.perf_counter()
    c0 = time.process_time()
    while time.perf_counter() - t0 < budget_s:
        OS.run(prob.model, X, p, prob.y, prob.I, sweep0=1 + n, n_sweeps=5, **kw)
        n += 5
    wall = time.perf_counter() - t0
    cpu = time.process_time() - c0
    return {"value": (prob.M + 1) * n / wall, "unit": "site-updates/s",
            "cores": max(1, round(cpu / wall)), "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"{n} sweeps of the same M={prob.M} window from its initial guess ({wall:.1f} s)"}


def _post_stats(traces, mask):
    """traces [chains][n][7] -> per sampled param: the sum over chains of the
    per-chain ESS, the pooled mean and its standard error from the spread of
    the chain means (chains are independent streams)."""
    import numpy as np
    from paper_1103_4887_amd import diag

    ess = np.array([diag.ess_columns(t[:, mask]) for t in traces]).sum(axis=0)
    cm = traces[:, :, mask].mean(axis=1)
    if len(cm) < 2:   # one chain: no spread of chain means to take
        return ess, cm.mean(axis=0), np.full(cm.shape[1], np.nan)
    return ess, cm.mean(axis=0), cm.std(axis=0, ddof=1) / np.sqrt(len(cm))


def hmc_vs_sweep(ctx, prob, chains: int, budget_s: float, equilibrate_s: float, L_steps: int = 20):
    """Parameter ESS per second of HMC and of the plain sweep on one dataset.

    The chains first equilibrate (untimed): `chains` chains of the batched
    sweep run for `equilibrate_s` seconds from the true path and parameters
    of the twin experiment.  Both samplers then start from these same states
    and get the same wall budget, their own warm-up included; ESS is summed
    over chains on the second half of each run.  HMC's warm-up is a pilot
    sweep run for the diagonal masses plus dual-averaging of the step size
    to 0.7 acceptance.
    """
    import numpy as np
    import torch

    import paper_1103_4887_amd as P
    from paper_1103_4887_amd import autotune
    from paper_1103_4887_amd import hmc as H

    spec = prob.model
    B = chains
    mask = [l for l in range(7) if (spec.p_mask >> l) & 1]
    w = P.widths_tensor(prob.w_state, prob.w_param)

    start = P.PackedBatch.pack([prob.X0] * B, [prob.p0] * B, [prob.y] * B, [prob.I] * B, list(range(B)), "fp32")
    # launch shape from the batch autotuner (a one-off per window set)
    shape = autotune.tune_batch(ctx, spec, start, w)
    # equilibration, not timed: distinct sweep counters from everything below
    n_eq = 0
    t_eq = time.perf_counter()
    while time.perf_counter() - t_eq < equilibrate_s:
        P.pimc_run_batch(ctx, spec, start, seed=prob.seed + 7, sweep0=n_eq, w=w, n_sweeps=20000)
        assert ctx.sync() == 0
        n_eq += 20000

    def fresh():
        return P.PackedBatch(offsets=start.offsets, X=start.X.clone(), p=start.p.clone(), y=start.y, I=start.I,
                             chain=start.chain, prec=start.prec)

    def batched(flags, seed_off):
        """`chains` chains of the batched sweep for the wall budget (a short
        run sizes the budgeted one); returns the run's record and its
        posterior statistics."""
        bm = fresh()
        t0 = time.perf_counter()
        try:
            P.pimc_run_batch(ctx, spec, bm, seed=prob.seed + seed_off, sweep0=0, w=w, n_sweeps=50, flags=flags)
            shape_f = shape
        except P._lib.PimcError as e:
            # the extended kernels (exact draws) take the shapes of at most 4
            # sites per thread and 256 threads: tune among those
            if e.status != P._lib.PIMC_ERR_UNSUPPORTED:
                raise
            shape_f = autotune.tune_batch(ctx, spec, bm, w, flags=flags)
            bm = fresh()
            t0 = time.perf_counter()
            P.pimc_run_batch(ctx, spec, bm, seed=prob.seed + seed_off, sweep0=0, w=w, n_sweeps=50, flags=flags)
        assert ctx.sync() == 0
        t_probe = time.perf_counter()
        P.pimc_run_batch(ctx, spec, bm, seed=prob.seed + seed_off, sweep0=50, w=w, n_sweeps=200, flags=flags)
        assert ctx.sync() == 0
        per_sweep = (time.perf_counter() - t_probe) / 200
        n_m = max(1000, int((budget_s - (time.perf_counter() - t0)) / per_sweep))
        stride = max(1, n_m // 20000)     # the trace is thinned on the host for the ESS estimate
        dev = bm.X.device
        sm = P.SweepStats(ptrace=torch.zeros((B, n_m, 7), dtype=torch.float64, device=dev),
                          acc=torch.zeros((B, P._lib.PIMC_NACC), dtype=torch.int64, device=dev))
        P.pimc_run_batch(ctx, spec, bm, seed=prob.seed + seed_off, sweep0=250, w=w, n_sweeps=n_m, stats=sm,
                         flags=flags)
        assert ctx.sync() == 0
        wall_m = time.perf_counter() - t0
        tr_m = sm.ptrace[:, n_m // 2::stride].cpu().numpy()
        del sm.ptrace
        ess_m, mean_m, mcse_m = _post_stats(tr_m, mask)
        acc_m = sm.acc.cpu().numpy()
        if shape_f is not shape:
            autotune.tune_batch(ctx, spec, start, w)   # back to the batch's own shape
        rec = {"chains": B, "launch": {"K": shape_f[0], "tiles": shape_f[1]}, "sweeps": n_m, "trace_stride": stride,
               "wall_s": wall_m, "us_per_sweep": per_sweep * 1e6,
               "site_updates_per_s": B * (prob.M + 1) * n_m / wall_m,
               "param_ess_per_s": float(ess_m.min() / wall_m),
               "param_ess_per_s_median": float(np.median(ess_m) / wall_m),
               "param_ess": [float(v) for v in ess_m],
               "accept_sites": float(acc_m[:, :2].sum() / (B * (prob.M + 1) * n_m))}
        return rec, ess_m.min() / wall_m, mean_m, mcse_m

    plain = P._lib.PIMC_STATES | P._lib.PIMC_PARAMS
    exact = plain | P._lib.PIMC_GIBBS
    rec_m, ess_rate_m, mean_m, mcse_m = batched(plain, 0)
    # the same with each parameter drawn from its exact conditional
    rec_g, ess_rate_g, mean_g, mcse_g = batched(exact, 5)

    # one chain (the benchmark's single-window launch, in its own autotuned
    # shape) from chain 0's equilibrated state, same budget
    x0, p0, _, _ = start.window(0)

    def single(flags, seed_off):
        win1 = P.Window(X=x0.clone(), p=p0.clone(), y=start.y[:prob.M + 1], I=start.I[:prob.M + 1], prec="fp32")
        autotune.tune(ctx, spec, win1, w)
        t0 = time.perf_counter()
        P.pimc_sweep(ctx, spec, win1, seed=prob.seed + seed_off, chain=0, sweep0=0, w=w, n_sweeps=200, flags=flags)
        assert ctx.sync() == 0
        per_sweep1 = (time.perf_counter() - t0) / 200
        n_1 = max(1000, int((budget_s - (time.perf_counter() - t0)) / per_sweep1))
        s1 = P.SweepStats.allocate(win1, n_1, moments=False)
        P.pimc_sweep(ctx, spec, win1, seed=prob.seed + seed_off, chain=0, sweep0=200, w=w, n_sweeps=n_1, stats=s1,
                     flags=flags)
        assert ctx.sync() == 0
        wall_1 = time.perf_counter() - t0
        stride1 = max(1, n_1 // 20000)
        tr_1 = s1.ptrace[n_1 // 2::stride1].cpu().numpy()[None]
        ess_1, _, _ = _post_stats(tr_1, mask)
        shape1 = autotune.tune(ctx, spec, win1, w)
        rec = {"launch": {"K": shape1[0], "tiles": shape1[1]}, "sweeps": n_1, "wall_s": wall_1,
               "us_per_sweep": per_sweep1 * 1e6, "param_ess_per_s": float(ess_1.min() / wall_1),
               "param_ess": [float(v) for v in ess_1]}
        return rec, ess_1.min() / wall_1

    rec_1, ess_rate_1 = single(plain, 3)
    rec_1g, ess_rate_1g = single(exact, 4)
    autotune.tune_batch(ctx, spec, start, w)   # the batch shape again (cached) for HMC's pilot run

    # HMC: pilot masses, step-size warm-up, then sampling in one graph-replayed call
    bh = fresh()
    t0 = time.perf_counter()
    minv = H.pilot_minv(ctx, spec, bh, w, seed=prob.seed + 1, sweeps=2000)
    tun = H.tune_eps(ctx, spec, bh, minv, seed=prob.seed + 2, L_steps=L_steps, warmup=200, eps0=0.01)
    t_probe = time.perf_counter()
    H.sample(ctx, spec, bh, tun, seed=prob.seed + 2, L_steps=L_steps, n=100, k0=200)
    per_prop = (time.perf_counter() - t_probe) / 100
    n_h = max(200, int((budget_s - (time.perf_counter() - t0)) / per_prop))
    sh = H.sample(ctx, spec, bh, tun, seed=prob.seed + 2, L_steps=L_steps, n=n_h, k0=300)
    wall_h = time.perf_counter() - t0
    tr_h = sh.ptrace.cpu().numpy()
    tr_h = tr_h[:, n_h // 2:]
    ess_h, mean_h, mcse_h = _post_stats(tr_h, mask)
    acc_h = sh.acc.cpu().numpy()

    z = np.abs(mean_h - mean_m) / np.sqrt(mcse_h ** 2 + mcse_m ** 2)
    zg = np.abs(mean_h - mean_g) / np.sqrt(mcse_h ** 2 + mcse_g ** 2)
    return {
        "dataset": f"HH M={prob.M}, dt={spec.dt} ms, all 7 params, FP32 sites + FP64 reductions",
        "chains": B, "start": f"true path and parameters, then {n_eq} sweeps of equilibration (untimed)",
        "budget_s": budget_s,
        "sweep": rec_m,
        "sweep_exact_draws": rec_g,
        "hmc": {"proposals": n_h, "leapfrog_steps": L_steps, "eps": tun.eps,
                "warmup_accept": tun.warmup_accept, "wall_s": wall_h, "us_per_proposal": per_prop * 1e6,
                "site_leapfrogs_per_s": B * (prob.M + 1) * L_steps * n_h / wall_h,
                "accept": float(acc_h[:, 0].sum() / (B * n_h)),
                "invalid": float(acc_h[:, 1].sum() / (B * n_h)),
                "param_ess_per_s": float(ess_h.min() / wall_h),
                "param_ess_per_s_median": float(np.median(ess_h) / wall_h),
                "param_ess": [float(v) for v in ess_h]},
        "single_chain_sweep": rec_1,
        "single_chain_exact_draws": rec_1g,
        "hmc_over_sweep_param_ess_per_s": float((ess_h.min() / wall_h) / ess_rate_m),
        "exact_draws_over_sweep_param_ess_per_s": float(ess_rate_g / ess_rate_m),
        "batched_over_single_param_ess_per_s": float(ess_rate_m / max(ess_rate_1, 1e-300)),
        "hmc_over_single_param_ess_per_s": float((ess_h.min() / wall_h) / max(ess_rate_1, 1e-300)),
        "single_exact_draws_over_single_param_ess_per_s": float(ess_rate_1g / max(ess_rate_1, 1e-300)),
        "equal_posterior_accuracy": {"max_z": float(z.max()), "within_3_mcse": bool((z <= 3.0).all()),
                                     "max_z_exact_draws_vs_hmc": float(zg.max()),
                                     "exact_draws_within_3_mcse": bool((zg <= 3.0).all()),
                                     "mcse": "spread of the chain means / sqrt(chains)",
                                     "mean_sweep": [float(v) for v in mean_m],
                                     "mean_exact_draws": [float(v) for v in mean_g],
                                     "mean_hmc": [float(v) for v in mean_h]},
    }


def _timed(stream, fn):
    """Run fn between two HIP events on `stream`; returns (seconds on the
    device clock, wall seconds, fn's result).  A short device-side delay is
    queued first, so that the host's work of issuing the call (Python
    marshalling, the launch) overlaps it, as it does in any caller that keeps
    the device busy: the events then time the device work of the call, all of
    it, without the idle gap of a device waiting for its first launch.  The
    delay (about 1 ms) also brings the device out of any idle clock state
    before the timed work starts.  The wall time (host clock, delay
    included) is reported beside it."""
    import torch

    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        torch.cuda._sleep(2000000)
    ev0.record(stream)
    r = fn()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return ev0.elapsed_time(ev1) / 1e3, wall, r


def _common(metric, value, unit, K, Wm, gpu_s, dtype, config):
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": K, "warmup": Wm,
            "ms_per_step": gpu_s * 1e3 / K, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": dtype, "data": "synthetic", "config": config}


def bench_batch(ctx, config: str, K: int, Wm: int, cpu_seconds: float):
    """The batched workload: 512 HH windows of uneven M (each with its own
    drive, noise and true parameters) swept together by one launch per call
    (the captured batch graph).  One step = one sweep of every window."""
    import torch

    import paper_1103_4887_amd as P
    from paper_1103_4887_amd import autotune
    import workloads as W

    cfg = W.CONFIGS[config]
    probs = W.config_batch(config, workers=host_cores())
    spec = probs[0].model
    B = len(probs)
    batch = P.PackedBatch.pack([q.X0 for q in probs], [q.p0 for q in probs], [q.y for q in probs],
                               [q.I for q in probs], list(range(B)), "fp32")
    w = P.widths_tensor(probs[0].w_state, probs[0].w_param)
    shape = autotune.tune_batch(ctx, spec, batch, w)
    P.pimc_run_batch(ctx, spec, batch, seed=cfg["data_seed"], sweep0=0, w=w, n_sweeps=max(Wm, 1))
    assert ctx.sync() == 0
    st = P.SweepStats(acc=torch.zeros((B, P._lib.PIMC_NACC), dtype=torch.int64, device=batch.X.device))
    stream = torch.cuda.current_stream()
    gpu_s, wall, _ = _timed(stream, lambda: P.pimc_run_batch(ctx, spec, batch, seed=cfg["data_seed"],
                                                              sweep0=max(Wm, 1), w=w, n_sweeps=K, stats=st))
    if ctx.sync() != 0:
        raise RuntimeError("device reported an error")
    sites = int(batch.offsets[-1])
    rate = sites * K / gpu_s
    acc = st.acc.cpu().numpy()
    achieved = SLOTS_PER_SITE_UPDATE * rate
    out = _common("path site-updates/s, uneven batch of HH windows, 1 GPU", rate, "site-updates/s", K, Wm,
                  gpu_s, "f32",
                  {"workload": f"{config}: {B} HH windows, M uniform in [{cfg['M_lo']}, {cfg['M_hi']}] "
                               f"({sites} sites), dt={spec.dt} ms, fp32 sites + f64 reductions, params mask "
                               f"0x{spec.p_mask:x}, one launch per call, {K} sweeps",
                   "windows": B, "sites": sites, "launch": {"K": shape[0], "tiles": shape[1]}})
    out["accept_rate"] = {"sites": float(acc[:, :2].sum() / (sites * K))}
    out["roofline"] = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_SLOTS_PER_S / 1e12,
                       "unit": "Tslot/s", "frac": achieved / PEAK_SLOTS_PER_S, "traffic": None,
                       "kernel": "sweep_kernel", "slots_per_site_update": SLOTS_PER_SITE_UPDATE,
                       "kernel_ms": gpu_s * 1e3, "wall_ms": wall * 1e3}
    if cpu_seconds > 0:
        # every host core on windows spread over the batch's range of M
        order = sorted(range(B), key=lambda i: probs[i].M)
        pick = [probs[order[(2 * j + 1) * B // (2 * host_cores())]] for j in range(host_cores())]
        out["cpu_baseline"] = cpu_baseline_ncore("sweep", pick, cpu_seconds)
        out["cpu_baseline"]["gpu_over_cpu"] = rate / out["cpu_baseline"]["value"]
    return out


def bench_hmc(ctx, config: str, K: int, Wm: int, cpu_seconds: float, ess_proposals: int = 2000):
    """HMC on the 64-chain workload: pilot masses and dual-averaged step size
    (untimed), then K proposals of L leapfrog steps replayed from one
    captured graph.  One step = one proposal of every chain.  The parameter
    ESS/s comes from a separate run of `ess_proposals` proposals (its own
    wall clock), long enough for the estimator."""
    import torch

    import paper_1103_4887_amd as P
    from paper_1103_4887_amd import autotune
    from paper_1103_4887_amd import hmc as H
    import workloads as W

    cfg = W.CONFIGS[config]
    prob = W.config_problem(config, init="truth")
    spec = prob.model
    B, L = cfg["chains"], cfg["leapfrog"]
    batch = P.PackedBatch.pack([prob.X0] * B, [prob.p0] * B, [prob.y] * B, [prob.I] * B, list(range(B)), "fp32")
    w = P.widths_tensor(prob.w_state, prob.w_param)
    autotune.tune_batch(ctx, spec, batch, w)
    minv = H.pilot_minv(ctx, spec, batch, w, seed=prob.seed + 1, sweeps=2000)
    tun = H.tune_eps(ctx, spec, batch, minv, seed=prob.seed + 2, L_steps=L, warmup=200, eps0=0.01)
    H.sample(ctx, spec, batch, tun, seed=prob.seed + 2, L_steps=L, n=max(Wm, 1), k0=200)
    stream = torch.cuda.current_stream()
    k1 = 200 + max(Wm, 1)
    gpu_s, wall, sh = _timed(stream, lambda: H.sample(ctx, spec, batch, tun, seed=prob.seed + 2, L_steps=L, n=K,
                                                      k0=k1))
    if ctx.sync() != 0:
        raise RuntimeError("device reported an error")
    sites = B * (prob.M + 1)
    rate = sites * L * K / gpu_s
    acc = sh.acc.cpu().numpy()
    out = _common("site-leapfrogs/s + param ESS/s, HMC, HH M=16384 x 64 chains, 1 GPU", rate, "site-leapfrogs/s",
                  K, Wm, gpu_s, "f32",
                  {"workload": f"{config}: HMC on {B} chains of the HH window M={prob.M}, dt={spec.dt} ms, "
                               f"{L} leapfrog steps per proposal, fp32 sites + f64 Hamiltonian, params mask "
                               f"0x{spec.p_mask:x}, {K} proposals",
                   "chains": B, "M": prob.M, "leapfrog_steps": L, "eps": tun.eps})
    out["accept_rate"] = float(acc[:, 0].sum() / (B * K))
    if ess_proposals > 0:
        mask = [l for l in range(7) if (spec.p_mask >> l) & 1]
        t0 = time.perf_counter()
        se = H.sample(ctx, spec, batch, tun, seed=prob.seed + 2, L_steps=L, n=ess_proposals, k0=k1 + K)
        wall_e = time.perf_counter() - t0
        ess, _, _ = _post_stats(se.ptrace.cpu().numpy()[:, ess_proposals // 2:], mask)
        out["param_ess_per_s"] = float(ess.min() / wall_e)
        out["param_ess"] = [float(v) for v in ess]
        out["param_ess_sample"] = (f"{ess_proposals} proposals of all {B} chains after the timed ones "
                                   f"({wall_e:.2f} s wall), ESS summed over chains on the second half")
    # per site-leapfrog the kernels move q, r (read and write) and read y, I
    out["roofline"] = {"bound": "hbm", "achieved": 72.0 * rate / 1e9, "peak": 8000.0, "unit": "GB/s",
                       "frac": 72.0 * rate / 8e12, "traffic": None, "kernel": "hmc_step_kernel",
                       "bytes_per_site_leapfrog": 72, "kernel_ms": gpu_s * 1e3, "wall_ms": wall * 1e3}
    if cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline_ncore("hmc", [prob], cpu_seconds, extra=(tun.eps, L, tun.minv))
        out["cpu_baseline"]["gpu_over_cpu"] = rate / out["cpu_baseline"]["value"]
    return out


def cpu_baseline_hmc(prob, tun, L, budget_s: float):
    """The oracle's HMC proposal, untouched, on one chain for a bounded number of proposals."""
    from oracle import hmc as OH

    X = prob.X0.copy()
    p = prob.p0.copy()
    n = 0
    t0 = time.perf_counter()
    c0 = time.process_time()
    while time.perf_counter() - t0 < budget_s:
        X, p, _, _ = OH.hmc_proposal(prob.model, X, p, prob.y, prob.I, seed=prob.seed, chain=0, k=n, e=tun.eps,
                                     L=L, minv_state=tun.minv[:4], minv_param=tun.minv[4:])
        n += 1
    wall = time.perf_counter() - t0
    cpu = time.process_time() - c0
    return {"value": (prob.M + 1) * L * n / wall, "unit": "site-leapfrogs/s",
            "cores": max(1, round(cpu / wall)), "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"{n} proposals of one M={prob.M} chain ({wall:.1f} s)"}


def bench_paper(args):
    """The paper-like run: Section 5.1's window (M = 8000 at 25 kHz, Ro = 100,
    Lorenz-driven twin data), its schedule (1e6 iterations, N_skip = 400,
    N_init = 5e5, annealing over 1e5 from beta0 = 0.01, f_acc = 0.23,
    alpha = 0.02; --steps shortens it proportionally) and the model checks of
    Section 6.  One step = one sweep of the whole window."""
    import paper_1103_4887_amd as P
    from paper_1103_4887_amd import replicate
    from workloads.paper_data import PAPER_RUN, make_paper_problem

    run = dict(PAPER_RUN)
    if args.steps:
        f = args.steps / run["sweeps"]
        run = {**run, "sweeps": args.steps, "n_init": int(run["n_init"] * f), "n_cool": max(1, int(run["n_cool"] * f)),
               "n_skip": max(1, int(run["n_skip"] * min(1.0, 10 * f)))}
    prob = make_paper_problem(M=run["M"], dt=run["dt"], Ro=run["Ro"])
    ctx = P.Context(0)
    t0 = time.perf_counter()
    out = replicate.run(ctx, prob, sweeps=run["sweeps"], n_init=run["n_init"], n_cool=run["n_cool"],
                        n_skip=run["n_skip"], beta0=run["beta0"], f_acc=run["f_acc"], alpha=run["alpha"],
                        verbose=True)
    wall = time.perf_counter() - t0
    ctx.close()
    sweeps = run["sweeps"]
    return {"metric": "paper-like run (Section 5.1 schedule) with the model checks of Section 6, 1 GPU",
            "value": (prob.M + 1) * sweeps / wall, "unit": "site-updates/s (whole run, wall clock)", "n_gpus": 1,
            "steps": sweeps, "ms_per_step": wall * 1e3 / sweeps, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"HH M={prob.M}, dt={prob.model.dt} ms, Ro={prob.model.Ro}, Lorenz-driven drive "
                                   f"({prob.meta['spikes']} spikes), uniform proposals, 7 parameters",
                       **run},
            "paper_gtx460_s_per_1e6_iterations": 683.0,
            "wall_s": wall, "result": out}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); multi-GPU runs are not part of this build",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1103_4887_amd as P
    from paper_1103_4887_amd import autotune
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    cpu_s = 0.0 if args.no_cpu_baseline else args.cpu_seconds
    if args.config == "paper":
        print(json.dumps(bench_paper(args)), flush=True)
        return
    if args.config in ("c4", "c5"):
        ctx = P.Context(0)
        if args.config == "c4":
            out = bench_batch(ctx, "c4", args.steps or 2000, args.warmup, cpu_s)
        else:
            out = bench_hmc(ctx, "c5", args.steps or 300, min(args.warmup, 50), cpu_s)
        ctx.close()
        print(json.dumps(out), flush=True)
        return
    cfg = W.CONFIGS[args.config]
    prob = W.config_problem(args.config)
    prec = cfg["prec"]
    ctx = P.Context(0)
    spec = prob.model
    win = P.Window.from_arrays(prob.X0, prob.p0, prob.y, prob.I, prec)
    w = P.widths_tensor(prob.w_state, prob.w_param)
    K, Wm = args.steps or 100000, args.warmup
    stream = torch.cuda.current_stream()
    if args.tiles < 0 and not args.tile:
        shape = autotune.tune(ctx, spec, win, w)
    else:
        ctx.set_tile(args.tile)
        ctx.set_tiles(max(args.tiles, 0))
        shape = (args.tile, max(args.tiles, 0), None)

    # warm-up (the library is prebuilt: nothing compiles here)
    P.pimc_sweep(ctx, spec, win, seed=prob.seed, chain=0, sweep0=0, w=w, n_sweeps=max(Wm, 1))
    assert ctx.sync() == 0
    stats = P.SweepStats.allocate(win, K, burn=Wm + K // 2, stride=args.nskip)
    gpu_s, wall, _ = _timed(stream, lambda: P.pimc_sweep(ctx, spec, win, seed=prob.seed, chain=0,
                                                         sweep0=max(Wm, 1), w=w, n_sweeps=K, stats=stats))
    st = ctx.sync()
    if st != 0:
        raise RuntimeError(f"device reported status {st}")
    sites = prob.M + 1
    rate = sites * K / gpu_s
    mask = [l for l in range(7) if (spec.p_mask >> l) & 1]
    acc = stats.acc.cpu().numpy()
    achieved = SLOTS_PER_SITE_UPDATE * rate
    out = {
        "metric": METRIC, "value": rate, "unit": "site-updates/s", "n_gpus": 1, "steps": K, "warmup": Wm,
        "ms_per_step": gpu_s * 1e3 / K, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if prec == "fp32" else "f64", "data": "synthetic",
        "config": {"workload": f"{args.config}: HH window M={prob.M}, dt={spec.dt} ms, {prec} sites + f64 "
                               f"reductions, params mask 0x{spec.p_mask:x}, 1 chain, {K} sweeps",
                   "M": prob.M, "sweeps": K, "chains": 1, "nskip": args.nskip,
                   "launch": {"K": shape[0], "tiles": shape[1]}},
        "param_ess_per_s": None,
        "param_ess_source": "not measured (the comparison of samplers was switched off)",
        "accept_rate": {"sites": float((acc[0] + acc[1]) / (sites * K)),
                        "params": [float(acc[2 + l] / K) for l in mask]},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_SLOTS_PER_S / 1e12,
                     "unit": "Tslot/s", "frac": achieved / PEAK_SLOTS_PER_S, "traffic": traffic_per_launch(shape, K),
                     "cus_occupied": max(1, shape[1]),
                     "frac_of_occupied_cus": achieved / (PEAK_SLOTS_PER_S / 256 * max(1, shape[1])),
                     "kernel": "sweep_kernel", "slots_per_site_update": SLOTS_PER_SITE_UPDATE,
                     "kernel_ms": gpu_s * 1e3, "wall_ms": wall * 1e3},
    }
    if args.cmp_seconds > 0:
        cmp = hmc_vs_sweep(ctx, W.config_problem(args.config, init="truth"), args.cmp_chains,
                           args.cmp_seconds, args.cmp_equilibrate)
        out["hmc_vs_sweep"] = cmp
        # the parameter ESS of this window's single chain needs tens of
        # seconds of sampling: it is the comparison's single-chain run (the
        # same window and launch shape), not the short timed run above
        one = cmp["single_chain_sweep"]
        out["param_ess_per_s"] = one["param_ess_per_s"]
        out["param_ess_source"] = (f"hmc_vs_sweep.single_chain_sweep: {one['sweeps']} sweeps of this window in "
                                   f"{one['wall_s']:.1f} s (Metropolis parameter moves); batched sweep and HMC "
                                   f"(64 chains) beside it")
        ex = cmp["single_chain_exact_draws"]
        out["param_ess_per_s_exact_draws"] = ex["param_ess_per_s"]
        out["param_ess_exact_draws_source"] = (f"hmc_vs_sweep.single_chain_exact_draws: {ex['sweeps']} sweeps of "
                                               f"this window in {ex['wall_s']:.1f} s, each parameter drawn from "
                                               f"its exact conditional (PIMC_GIBBS)")
    if cpu_s > 0:
        out["cpu_baseline"] = cpu_baseline(prob, cpu_s)
        out["cpu_baseline"]["gpu_over_cpu"] = rate / out["cpu_baseline"]["value"]
    if args.config == "c2" and args.sub_blocks:
        # short measurements of the batched and HMC workloads, so that every
        # run of the default benchmark also records them
        out["c4_batch"] = bench_batch(ctx, "c4", 200, 20, cpu_s)
        out["c5_hmc"] = bench_hmc(ctx, "c5", 30, 10, cpu_s, ess_proposals=2000)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
