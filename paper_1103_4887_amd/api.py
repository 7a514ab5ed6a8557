"""Python binding of libpimc with the C ABI's names.

Every function marshals torch tensors (device memory) and the current HIP
stream into the C calls; all arithmetic of the method runs in the library's
kernels.  A model description is any object with the attributes of the
pimc_model struct (dt, Ro, Rd, beta, gates = ((V_a, dV_a, tau0, tau1) for
m, h, n), x_lo, x_hi, p_lo, p_hi, p_mask, proposal).
"""

from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L

DTYPES = {"fp64": torch.float64, "fp32": torch.float32}
PRECS = {"fp64": L.PIMC_FP64, "fp32": L.PIMC_FP32}


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("libpimc takes device tensors")
    if not t.is_contiguous():
        raise ValueError("libpimc takes contiguous tensors")
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


_MODEL_CACHE: dict = {}


def model_struct(spec) -> L.Model:
    """The pimc_model of a model description.  Hashable (immutable)
    descriptions are converted once and the struct is reused by later calls
    (the library only reads it), which keeps the per-call cost of the
    binding small; treat the returned struct as read-only."""
    try:
        m = _MODEL_CACHE.get(spec)
    except TypeError:          # not hashable: convert every time
        return _model_struct(spec)
    if m is None:
        m = _model_struct(spec)
        if len(_MODEL_CACHE) > 256:
            _MODEL_CACHE.clear()
        _MODEL_CACHE[spec] = m
    return m


def _model_struct(spec) -> L.Model:
    m = L.Model()
    m.dt = float(spec.dt)
    m.Ro = float(spec.Ro)
    for i in range(4):
        m.Rd[i] = float(spec.Rd[i])
        m.x_lo[i] = float(spec.x_lo[i])
        m.x_hi[i] = float(spec.x_hi[i])
    m.beta = float(spec.beta)
    for g in range(3):
        Va, dVa, t0, t1 = spec.gates[g]
        m.Va[g], m.dVa[g], m.tau0[g], m.tau1[g] = float(Va), float(dVa), float(t0), float(t1)
    for l in range(7):
        m.p_lo[l] = float(spec.p_lo[l])
        m.p_hi[l] = float(spec.p_hi[l])
    m.p_mask = int(spec.p_mask)
    m.proposal = L.PIMC_PROP_UNIFORM if spec.proposal == "uniform" else L.PIMC_PROP_GAUSS
    k_lo = getattr(spec, "k_lo", None)
    k_hi = getattr(spec, "k_hi", None)
    for i in range(12):
        m.k_lo[i] = float(k_lo[i]) if k_lo is not None else -1e300
        m.k_hi[i] = float(k_hi[i]) if k_hi is not None else 1e300
    m.k_mask = int(getattr(spec, "k_mask", 0))
    return m


class Context:
    """A libpimc context on one HIP device (owns only its small workspace)."""

    def __init__(self, device: int = 0):
        self.lib = L.load()
        self.device = device
        h = C.c_void_p()
        L.check(self.lib.pimc_ctx_create(C.byref(h), device), "pimc_ctx_create")
        self.h = h

    def close(self):
        if self.h:
            self.lib.pimc_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_tile(self, K: int):
        L.check(self.lib.pimc_set_sweep_tile(self.h, int(K)), "pimc_set_sweep_tile")

    def set_tiles(self, T: int):
        L.check(self.lib.pimc_set_sweep_tiles(self.h, int(T)), "pimc_set_sweep_tiles")

    def sync(self, stream=None) -> int:
        """Wait for the stream; returns the deferred device status (0 = ok)."""
        return int(self.lib.pimc_sync(self.h, _stream(stream)))


@dataclass
class Window:
    """Device-resident window: X [M+1][4], p [7] FP64, y, I [M+1]; kin, if
    set, [12] FP64 Table 1 constants of the window (order (m, h, n) x
    (V_a, dV_a, tau0, tau1)) that replace the model's and that PIMC_KINETIC
    samples."""

    X: torch.Tensor
    p: torch.Tensor
    y: torch.Tensor
    I: torch.Tensor
    prec: str
    kin: Optional[torch.Tensor] = None

    @property
    def M(self) -> int:
        return self.X.shape[0] - 1

    @staticmethod
    def from_arrays(X, p, y, I, prec: str = "fp32", device: str = "cuda") -> "Window":
        dt = DTYPES[prec]
        return Window(X=torch.as_tensor(np.asarray(X), dtype=dt, device=device).contiguous(),
                      p=torch.as_tensor(np.asarray(p), dtype=torch.float64, device=device).contiguous(),
                      y=torch.as_tensor(np.asarray(y), dtype=dt, device=device).contiguous(),
                      I=torch.as_tensor(np.asarray(I), dtype=dt, device=device).contiguous(),
                      prec=prec)

    def path_struct(self) -> L.Path:
        pa = L.Path()
        pa.M = self.M
        pa.prec = PRECS[self.prec]
        pa.X = _ptr(self.X)
        pa.p = _ptr(self.p)
        pa.y = _ptr(self.y)
        pa.I = _ptr(self.I)
        pa.kin = _ptr(self.kin)
        return pa


@dataclass
class SweepStats:
    sum: Optional[torch.Tensor] = None
    sumsq: Optional[torch.Tensor] = None
    xref: Optional[torch.Tensor] = None
    ptrace: Optional[torch.Tensor] = None
    acc: Optional[torch.Tensor] = None
    burn: int = 0
    stride: int = 1
    batch: Optional[torch.Tensor] = None    # [nbatch][sites][4] per-batch sums
    kacc: Optional[torch.Tensor] = None     # [12] int64 accepted moves of the Table 1 constants

    @staticmethod
    def allocate(win: Window, n_sweeps: int, burn: int = 0, moments: bool = True, trace: bool = True,
                 stride: int = 1, nbatch: int = 0):
        dev = win.X.device
        st = SweepStats(burn=burn, stride=stride)
        if moments:
            st.sum = torch.zeros((win.M + 1, 4), dtype=torch.float64, device=dev)
            st.sumsq = torch.zeros_like(st.sum)
            st.xref = win.X.clone()
            if nbatch > 0:
                st.batch = torch.zeros((nbatch, win.M + 1, 4), dtype=torch.float64, device=dev)
        if trace:
            st.ptrace = torch.zeros((n_sweeps, 7), dtype=torch.float64, device=dev)
        st.acc = torch.zeros(L.PIMC_NACC, dtype=torch.int64, device=dev)
        return st

    def struct(self) -> L.Stats:
        s = L.Stats()
        s.sum, s.sumsq, s.xref = _ptr(self.sum), _ptr(self.sumsq), _ptr(self.xref)
        s.ptrace, s.acc = _ptr(self.ptrace), _ptr(self.acc)
        s.burn = int(self.burn)
        s.stride = int(self.stride)
        s.batch = _ptr(self.batch)
        s.nbatch = int(self.batch.shape[0]) if self.batch is not None else 0
        s.kacc = _ptr(self.kacc)
        return s


@dataclass
class SweepDebug:
    xprop: Optional[torch.Tensor] = None
    dA: Optional[torch.Tensor] = None
    accept: Optional[torch.Tensor] = None
    pprop: Optional[torch.Tensor] = None
    pdA: Optional[torch.Tensor] = None
    paccept: Optional[torch.Tensor] = None
    kprop: Optional[torch.Tensor] = None
    kdA: Optional[torch.Tensor] = None
    kaccept: Optional[torch.Tensor] = None

    @staticmethod
    def allocate(win: Window, sites: bool = True, kinetic: bool = False, params: Optional[bool] = None):
        """Record of the last sweep: the sites (sites=True), the parameter
        moves (params; by default with the sites) and the kinetic constants
        (kinetic=True).  Calls with PIMC_KINETIC or PIMC_GIBBS record the
        parameters and kinetic constants only."""
        dev = win.X.device
        nan = float("nan")
        d = SweepDebug()
        if sites:
            d.xprop = torch.full_like(win.X, nan)
            d.dA = torch.full((win.M + 1,), nan, dtype=torch.float64, device=dev)
            d.accept = torch.zeros(win.M + 1, dtype=torch.uint8, device=dev)
        if sites if params is None else params:
            d.pprop = torch.full((7,), nan, dtype=torch.float64, device=dev)
            d.pdA = torch.full((7,), nan, dtype=torch.float64, device=dev)
            d.paccept = torch.zeros(7, dtype=torch.uint8, device=dev)
        if kinetic:
            d.kprop = torch.full((12,), nan, dtype=torch.float64, device=dev)
            d.kdA = torch.full((12,), nan, dtype=torch.float64, device=dev)
            d.kaccept = torch.zeros(12, dtype=torch.uint8, device=dev)
        return d

    def struct(self) -> L.Debug:
        d = L.Debug()
        d.xprop, d.dA, d.accept = _ptr(self.xprop), _ptr(self.dA), _ptr(self.accept)
        d.pprop, d.pdA, d.paccept = _ptr(self.pprop), _ptr(self.pdA), _ptr(self.paccept)
        d.kprop, d.kdA, d.kaccept = _ptr(self.kprop), _ptr(self.kdA), _ptr(self.kaccept)
        return d


def _rng(seed: int, chain: int, sweep0: int) -> L.Rng:
    r = L.Rng()
    r.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    r.chain = int(chain) & 0xFFFFFFFF
    r.sweep0 = int(sweep0)
    return r


def widths_tensor(w_state: Sequence[float], w_param: Sequence[float], device="cuda") -> torch.Tensor:
    return torch.tensor(list(w_state) + list(w_param), dtype=torch.float64, device=device)


def pimc_action(ctx: Context, spec, win: Window, out3: Optional[torch.Tensor] = None, stream=None):
    if out3 is None:
        out3 = torch.empty(3, dtype=torch.float64, device=win.X.device)
    m, pa = model_struct(spec), win.path_struct()
    L.check(ctx.lib.pimc_action(ctx.h, C.byref(m), C.byref(pa), _ptr(out3), _stream(stream)), "pimc_action")
    return out3


def pimc_model_errors(ctx: Context, spec, win: Window, esum: torch.Tensor, esq: torch.Tensor, stream=None):
    """Add the model and observation errors of the window's current path to
    esum / esq ([M][5] FP64 device tensors)."""
    m, pa = model_struct(spec), win.path_struct()
    L.check(ctx.lib.pimc_model_errors(ctx.h, C.byref(m), C.byref(pa), _ptr(esum), _ptr(esq), _stream(stream)),
            "pimc_model_errors")


def pimc_forecast(ctx: Context, spec, x0: torch.Tensor, p: torch.Tensor, I: torch.Tensor, N: int, *,
                  noise: float = 0.0, seed: int = 0, member0: int = 0, kin: Optional[torch.Tensor] = None,
                  out: Optional[torch.Tensor] = None, stream=None):
    """Forecast ensemble: x0 [B][4], p [B][7], drive I [N+1] (FP64 device
    tensors); returns [B][N+1][4]."""
    B = int(x0.shape[0])
    if out is None:
        out = torch.empty((B, N + 1, 4), dtype=torch.float64, device=x0.device)
    m = model_struct(spec)
    L.check(ctx.lib.pimc_forecast(ctx.h, C.byref(m), B, _ptr(x0), _ptr(p), _ptr(kin), _ptr(I), int(N),
                                  float(noise), int(seed) & 0xFFFFFFFFFFFFFFFF, int(member0), _ptr(out),
                                  _stream(stream)), "pimc_forecast")
    return out


def pimc_action_noalloc(spec, win: Window, out3: torch.Tensor, stream=None):
    """pimc_action through the library's fixed workspace: allocates nothing
    (out3 is the caller's [3] FP64 device tensor)."""
    m, pa = model_struct(spec), win.path_struct()
    L.check(L.load().pimc_action_noalloc(C.byref(m), C.byref(pa), _ptr(out3), _stream(stream)),
            "pimc_action_noalloc")
    return out3


def pimc_grad(ctx: Context, spec, win: Window, gX: Optional[torch.Tensor] = None,
              gp: Optional[torch.Tensor] = None, stream=None):
    if gX is None:
        gX = torch.empty_like(win.X)
    if gp is None:
        gp = torch.empty(7, dtype=torch.float64, device=win.X.device)
    m, pa = model_struct(spec), win.path_struct()
    L.check(ctx.lib.pimc_grad(ctx.h, C.byref(m), C.byref(pa), _ptr(gX), _ptr(gp), _stream(stream)), "pimc_grad")
    return gX, gp


def pimc_sweep(ctx: Context, spec, win: Window, *, seed: int, chain: int, sweep0: int, w: torch.Tensor,
               n_sweeps: int, flags: int = L.PIMC_STATES | L.PIMC_PARAMS,
               stats: Optional[SweepStats] = None, debug: Optional[SweepDebug] = None, stream=None):
    m, pa = model_struct(spec), win.path_struct()
    st = C.byref(stats.struct()) if stats is not None else None
    db = C.byref(debug.struct()) if debug is not None else None
    L.check(ctx.lib.pimc_sweep(ctx.h, C.byref(m), C.byref(pa), _rng(seed, chain, sweep0), _ptr(w),
                               int(n_sweeps), int(flags), st, db, _stream(stream)), "pimc_sweep")


def pimc_param_update(ctx: Context, spec, win: Window, *, seed: int, chain: int, sweep0: int,
                      w: torch.Tensor, debug: Optional[SweepDebug] = None, stream=None):
    m, pa = model_struct(spec), win.path_struct()
    db = C.byref(debug.struct()) if debug is not None else None
    L.check(ctx.lib.pimc_param_update(ctx.h, C.byref(m), C.byref(pa), _rng(seed, chain, sweep0), _ptr(w),
                                      db, _stream(stream)), "pimc_param_update")


@dataclass
class InitPhase:
    """Device state of the initialization phase (annealing and step-size
    adjustment, see pimc_init_phase in include/pimc.h); consecutive calls of
    pimc_sweep_init with the same object continue the phase."""

    beta0: float
    n_cool: int
    n_init: int
    n_skip: int
    f_acc: float
    alpha: float
    beta: torch.Tensor         # [1] FP64
    site_scale: torch.Tensor   # [M+1] FP64
    w_param: torch.Tensor      # [7] FP64
    cnt_site: torch.Tensor     # [M+1] int32
    cnt_param: torch.Tensor    # [7] int32

    @staticmethod
    def start(win: "Window", w_param, *, beta0: float, n_cool: int, n_init: int, n_skip: int,
              f_acc: float = 0.23, alpha: float = 0.02) -> "InitPhase":
        dev = win.X.device
        return InitPhase(beta0=beta0, n_cool=n_cool, n_init=n_init, n_skip=n_skip, f_acc=f_acc, alpha=alpha,
                         beta=torch.full((1,), float(beta0), dtype=torch.float64, device=dev),
                         site_scale=torch.ones(win.M + 1, dtype=torch.float64, device=dev),
                         w_param=torch.as_tensor(np.asarray(w_param, dtype=np.float64), device=dev).clone(),
                         cnt_site=torch.zeros(win.M + 1, dtype=torch.int32, device=dev),
                         cnt_param=torch.zeros(7, dtype=torch.int32, device=dev))

    def struct(self) -> L.InitPhase:
        s = L.InitPhase()
        s.beta0, s.n_cool, s.n_init, s.n_skip = float(self.beta0), int(self.n_cool), int(self.n_init), int(self.n_skip)
        s.f_acc, s.alpha = float(self.f_acc), float(self.alpha)
        s.beta, s.site_scale, s.w_param = _ptr(self.beta), _ptr(self.site_scale), _ptr(self.w_param)
        s.cnt_site, s.cnt_param = _ptr(self.cnt_site), _ptr(self.cnt_param)
        return s


def pimc_sweep_init(ctx: Context, spec, win: Window, *, seed: int, chain: int, sweep0: int, w: torch.Tensor,
                    n_sweeps: int, init: InitPhase, flags: int = L.PIMC_STATES | L.PIMC_PARAMS,
                    stats: Optional[SweepStats] = None, stream=None):
    """Sweeps with the initialization phase of Section 4.2 (see InitPhase)."""
    m, pa = model_struct(spec), win.path_struct()
    st = C.byref(stats.struct()) if stats is not None else None
    ip = init.struct()
    L.check(ctx.lib.pimc_sweep_init(ctx.h, C.byref(m), C.byref(pa), _rng(seed, chain, sweep0), _ptr(w),
                                    int(n_sweeps), int(flags), C.byref(ip), st, _stream(stream)), "pimc_sweep_init")


@dataclass
class PackedBatch:
    """Windows packed end to end: X [S][4], y, I [S], p [B][7], chain [B]."""

    offsets: np.ndarray      # host int64 [B+1]
    X: torch.Tensor
    p: torch.Tensor
    y: torch.Tensor
    I: torch.Tensor
    chain: torch.Tensor
    prec: str

    @property
    def B(self) -> int:
        return len(self.offsets) - 1

    @staticmethod
    def pack(Xs, ps, ys, Is, chains, prec: str = "fp32", device: str = "cuda") -> "PackedBatch":
        dt = DTYPES[prec]
        sizes = [len(X) for X in Xs]
        off = np.zeros(len(Xs) + 1, dtype=np.int64)
        off[1:] = np.cumsum(sizes)
        return PackedBatch(
            offsets=off,
            X=torch.as_tensor(np.concatenate(Xs), dtype=dt, device=device).contiguous(),
            p=torch.as_tensor(np.stack(ps), dtype=torch.float64, device=device).contiguous(),
            y=torch.as_tensor(np.concatenate(ys), dtype=dt, device=device).contiguous(),
            I=torch.as_tensor(np.concatenate(Is), dtype=dt, device=device).contiguous(),
            chain=torch.as_tensor(np.asarray(chains, dtype=np.uint32).view(np.int32), device=device).contiguous(),
            prec=prec)

    def struct(self):
        b = L.Batch()
        b.B = self.B
        b.prec = PRECS[self.prec]
        self._off = (C.c_int64 * len(self.offsets))(*[int(v) for v in self.offsets])
        b.offsets = C.cast(self._off, C.POINTER(C.c_int64))
        b.X, b.p, b.y, b.I, b.chain = _ptr(self.X), _ptr(self.p), _ptr(self.y), _ptr(self.I), _ptr(self.chain)
        return b

    def window(self, w: int):
        a, b = int(self.offsets[w]), int(self.offsets[w + 1])
        return self.X[a:b], self.p[w], self.y[a:b], self.I[a:b]


def pimc_run_batch(ctx: Context, spec, batch: PackedBatch, *, seed: int, sweep0: int, w: torch.Tensor,
                   n_sweeps: int, flags: int = L.PIMC_STATES | L.PIMC_PARAMS,
                   stats: Optional[SweepStats] = None, stream=None):
    m = model_struct(spec)
    b = batch.struct()
    st = None
    if stats is not None:
        bs = L.BatchStats()
        bs.sum, bs.sumsq, bs.xref = _ptr(stats.sum), _ptr(stats.sumsq), _ptr(stats.xref)
        bs.ptrace, bs.acc, bs.burn = _ptr(stats.ptrace), _ptr(stats.acc), int(stats.burn)
        bs.stride = int(stats.stride)
        bs.batch = _ptr(stats.batch)
        bs.nbatch = int(stats.batch.shape[0]) if stats.batch is not None else 0
        st = C.byref(bs)
    L.check(ctx.lib.pimc_run_batch(ctx.h, C.byref(m), C.byref(b), int(seed), int(sweep0), _ptr(w),
                                   int(n_sweeps), int(flags), st, _stream(stream)), "pimc_run_batch")


@dataclass
class HmcStats:
    acc: Optional[torch.Tensor] = None      # [B][10] int64
    ptrace: Optional[torch.Tensor] = None   # [B][n][7]
    dH: Optional[torch.Tensor] = None       # [B][n]
    # trajectory of the last proposal (all four or none)
    traj_q: Optional[torch.Tensor] = None   # [L+1][S][4] positions q(s)
    traj_r: Optional[torch.Tensor] = None   # [L+1][S][4] momenta r(s+1/2), r(L) last
    traj_p: Optional[torch.Tensor] = None   # [L+1][B][7] parameters p(s)
    traj_rp: Optional[torch.Tensor] = None  # [L+2][B][7] rp(0), rp(s-1/2), rp(L)

    @staticmethod
    def allocate(B: int, n: int, device="cuda", trajectory: Optional[PackedBatch] = None, L_steps: int = 0):
        st = HmcStats(acc=torch.zeros((B, L.PIMC_NACC), dtype=torch.int64, device=device),
                      ptrace=torch.zeros((B, n, 7), dtype=torch.float64, device=device),
                      dH=torch.zeros((B, n), dtype=torch.float64, device=device))
        if trajectory is not None:
            S = int(trajectory.offsets[-1])
            dt = DTYPES[trajectory.prec]
            st.traj_q = torch.full((L_steps + 1, S, 4), float("nan"), dtype=dt, device=device)
            st.traj_r = torch.full_like(st.traj_q, float("nan"))
            st.traj_p = torch.full((L_steps + 1, B, 7), float("nan"), dtype=torch.float64, device=device)
            st.traj_rp = torch.full((L_steps + 2, B, 7), float("nan"), dtype=torch.float64, device=device)
        return st

    def struct(self) -> L.HmcStats:
        s = L.HmcStats()
        s.acc, s.ptrace, s.dH = _ptr(self.acc), _ptr(self.ptrace), _ptr(self.dH)
        s.traj_q, s.traj_r = _ptr(self.traj_q), _ptr(self.traj_r)
        s.traj_p, s.traj_rp = _ptr(self.traj_p), _ptr(self.traj_rp)
        return s


def pimc_hmc(ctx: Context, spec, batch: PackedBatch, *, seed: int, k0: int, eps: float, L_steps: int,
             minv: Sequence[float], n_proposals: int, stats: Optional[HmcStats] = None, stream=None):
    """Hybrid Monte Carlo proposals for every window of a packed batch."""
    m = model_struct(spec)
    b = batch.struct()
    mv = (C.c_double * 11)(*[float(v) for v in minv])
    st = C.byref(stats.struct()) if stats is not None else None
    L.check(ctx.lib.pimc_hmc(ctx.h, C.byref(m), C.byref(b), int(seed), int(k0), float(eps), int(L_steps), mv,
                             int(n_proposals), st, _stream(stream)), "pimc_hmc")
