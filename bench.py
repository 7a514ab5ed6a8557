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

# VALU lane-slots the method needs per FP32-mode site update, counted from
# its arithmetic (see the per-unit table of the design notes): Philox 1.25
# blocks, Box-Muller, F(x') and dF, local dA, FP64 log for the decision,
# the parameter sufficient-statistic link, neighbour exchange.
SLOTS_PER_SITE_UPDATE = 560
PEAK_SLOTS_PER_S = 256 * 4 * 16 * 2.4e9     # CUs x SIMDs x lanes x clock


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100000)
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tile", type=int, default=0, help="sites per thread (0: autotune)")
    ap.add_argument("--tiles", type=int, default=-1, help="time tiles per window (-1: autotune)")
    ap.add_argument("--nskip", type=int, default=10, help="path moments every nskip-th sweep (N_skip)")
    return ap.parse_args()


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
            "cores": max(1, round(cpu / wall)), "kind": "oracle",
            "sample": f"{n} sweeps of the same M={prob.M} window from its initial guess ({wall:.1f} s)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); multi-GPU runs are not part of this build",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1103_4887_amd as P
    from paper_1103_4887_amd import autotune, diag
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    cfg = W.CONFIGS[args.config]
    prob = W.config_problem(args.config)
    prec = cfg["prec"]
    ctx = P.Context(0)
    spec = prob.model
    win = P.Window.from_arrays(prob.X0, prob.p0, prob.y, prob.I, prec)
    w = P.widths_tensor(prob.w_state, prob.w_param)
    K, Wm = args.steps, args.warmup
    stream = torch.cuda.current_stream()
    if args.tiles < 0 and not args.tile:
        shape = autotune.tune(ctx, spec, win, w)
    else:
        ctx.set_tile(args.tile)
        ctx.set_tiles(max(args.tiles, 0))
        shape = (args.tile, max(args.tiles, 0), None)

    # warm-up (also compiles nothing: the library is prebuilt)
    P.pimc_sweep(ctx, spec, win, seed=prob.seed, chain=0, sweep0=0, w=w, n_sweeps=max(Wm, 1))
    assert ctx.sync() == 0
    stats = P.SweepStats.allocate(win, K, burn=Wm + K // 2, stride=args.nskip)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    P.pimc_sweep(ctx, spec, win, seed=prob.seed, chain=0, sweep0=max(Wm, 1), w=w, n_sweeps=K, stats=stats)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = ctx.sync()
    if st != 0:
        raise RuntimeError(f"device reported status {st}")
    gpu_s = ev0.elapsed_time(ev1) / 1e3
    sites = prob.M + 1
    rate = sites * K / gpu_s

    tr = stats.ptrace.cpu().numpy()
    post = tr[K // 2:]
    mask = [l for l in range(7) if (spec.p_mask >> l) & 1]
    ess = diag.ess_columns(post[:, mask])
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
        "param_ess_per_s": float(ess.min() / gpu_s),
        "param_ess_per_s_median": float(np.median(ess) / gpu_s),
        "param_ess": [float(v) for v in ess],
        "accept_rate": {"sites": float((acc[0] + acc[1]) / (sites * K)),
                        "params": [float(acc[2 + l] / K) for l in mask]},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_SLOTS_PER_S / 1e12,
                     "unit": "Tslot/s", "frac": achieved / PEAK_SLOTS_PER_S, "traffic": None,
                     "cus_occupied": max(1, shape[1]),
                     "frac_of_occupied_cus": achieved / (PEAK_SLOTS_PER_S / 256 * max(1, shape[1])),
                     "kernel": "sweep_kernel", "slots_per_site_update": SLOTS_PER_SITE_UPDATE,
                     "kernel_ms": gpu_s * 1e3, "wall_ms": wall * 1e3},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_seconds)
        out["cpu_baseline"]["gpu_over_cpu"] = rate / out["cpu_baseline"]["value"]
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
