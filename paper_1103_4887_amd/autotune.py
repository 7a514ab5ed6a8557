"""Launch-shape autotuner for the sweep kernel (single windows and batches).

The sweep's result does not depend on its launch shape (random numbers are
addressed by site and sweep; the shape only changes the rounding order of the
parameter statistics), so the shape is a pure performance choice: sites per
thread K and time tiles T per window.  The tuner times a short run of every
candidate on a scratch copy of the window and keeps the fastest; results are
cached per (M, precision, parameter flags) for the process.
"""

from __future__ import annotations

from typing import Dict, Iterable, Optional, Tuple

import torch

from . import _lib as L
from .api import Context, Window, pimc_sweep

_CACHE: Dict[Tuple[int, str, int], Tuple[int, int, float]] = {}


def candidates(M: int, prec: str, narrow: bool = False) -> Iterable[Tuple[int, int]]:
    """(K, T) pairs worth timing; K = 0 / T = 0 mean the library's own choice.
    narrow: only shapes of at most 256 threads per workgroup (the automatic
    choice and time tiles), the ones the extended kernels run in."""
    yield (0, 0)
    if prec == "fp64":
        return
    if not narrow:
        for K in (4, 8, 16):
            yield (K, 1)
    for T in (2, 4, 8, 16, 32, 64, 128):
        if M // T >= 256:
            yield (0, T)
        if M // T >= 128:
            yield (2, T)


def tune(ctx: Context, spec, win: Window, w: torch.Tensor, *, flags: int = L.PIMC_STATES | L.PIMC_PARAMS,
         sweeps: int = 200, seed: int = 12345, verbose: bool = False, narrow: bool = False) -> Tuple[int, int, float]:
    """Pick (K, T) for this window; applies it to ctx and returns (K, T, us_per_sweep).
    narrow: choose among the shapes the extended kernels run in (initialization
    phase, kinetic constants)."""
    key = (win.M, win.prec, flags, narrow)
    if key in _CACHE:
        K, T, us = _CACHE[key]
        ctx.set_tile(K)
        ctx.set_tiles(T)
        return K, T, us
    best: Optional[Tuple[int, int, float]] = None
    scratch = Window(X=win.X.clone(), p=win.p.clone(), y=win.y, I=win.I, prec=win.prec)
    for K, T in candidates(win.M, win.prec, narrow):
        ctx.set_tile(K)
        ctx.set_tiles(T)
        try:
            pimc_sweep(ctx, spec, scratch, seed=seed, chain=0, sweep0=0, w=w, n_sweeps=10, flags=flags)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            pimc_sweep(ctx, spec, scratch, seed=seed, chain=0, sweep0=10, w=w, n_sweeps=sweeps, flags=flags)
            e1.record()
            torch.cuda.synchronize()
        except L.PimcError:
            continue
        if ctx.sync() != 0:
            continue
        us = e0.elapsed_time(e1) * 1e3 / sweeps
        if verbose:
            print(f"autotune M={win.M} {win.prec} K={K} T={T}: {us:.2f} us/sweep", flush=True)
        if best is None or us < best[2]:
            best = (K, T, us)
    if best is None:
        raise RuntimeError("no launch shape of the sweep kernel runs this window")
    _CACHE[key] = best
    ctx.set_tile(best[0])
    ctx.set_tiles(best[1])
    return best


_BCACHE: Dict[Tuple, Tuple[int, int, float]] = {}


def batch_candidates(sizes, prec: str) -> Iterable[Tuple[int, int]]:
    """(K, T) pairs for a batch: one workgroup per window with each K, and
    time tiles for batches of equal windows long enough to be cut (the
    library tiles a batch only when every window needs the same number of
    tiles; windows of different lengths run one workgroup each)."""
    yield (0, 1)
    for K in ((4,) if prec == "fp64" else (4, 8, 16)):
        yield (K, 1)
    if prec == "fp64" or min(sizes) != max(sizes):
        return
    lo = int(min(sizes))
    for T in (2, 4, 8, 16):
        if lo // T >= 256 and len(sizes) * T <= 4096:
            yield (0, T)
        if lo // T >= 128 and len(sizes) * T <= 4096:
            yield (2, T)


def tune_batch(ctx: Context, spec, batch, w: torch.Tensor, *, flags: int = L.PIMC_STATES | L.PIMC_PARAMS,
               sweeps: int = 50, seed: int = 12345, verbose: bool = False) -> Tuple[int, int, float]:
    """Pick (K, T) for a packed batch; applies it to ctx and returns (K, T, us_per_sweep)."""
    from .api import PackedBatch, pimc_run_batch

    sizes = [int(batch.offsets[i + 1] - batch.offsets[i] - 1) for i in range(batch.B)]
    key = (tuple(sizes), batch.prec, flags)
    if key in _BCACHE:
        K, T, us = _BCACHE[key]
        ctx.set_tile(K)
        ctx.set_tiles(T)
        return K, T, us
    scratch = PackedBatch(offsets=batch.offsets, X=batch.X.clone(), p=batch.p.clone(), y=batch.y, I=batch.I,
                          chain=batch.chain, prec=batch.prec)
    best: Optional[Tuple[int, int, float]] = None
    for K, T in batch_candidates(sizes, batch.prec):
        ctx.set_tile(K)
        ctx.set_tiles(T)
        try:
            pimc_run_batch(ctx, spec, scratch, seed=seed, sweep0=0, w=w, n_sweeps=5, flags=flags)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            pimc_run_batch(ctx, spec, scratch, seed=seed, sweep0=5, w=w, n_sweeps=sweeps, flags=flags)
            e1.record()
            torch.cuda.synchronize()
        except L.PimcError:
            continue
        if ctx.sync() != 0:
            continue
        us = e0.elapsed_time(e1) * 1e3 / sweeps
        if verbose:
            print(f"autotune batch B={batch.B} {batch.prec} K={K} T={T}: {us:.2f} us/sweep", flush=True)
        if best is None or us < best[2]:
            best = (K, T, us)
    if best is None:
        raise RuntimeError("no launch shape of the sweep kernel runs this batch")
    _BCACHE[key] = best
    ctx.set_tile(best[0])
    ctx.set_tiles(best[1])
    return best
