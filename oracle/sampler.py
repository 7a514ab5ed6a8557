"""Red-black Metropolis sweep with sequential parameter moves (oracle, FP64).

One sweep k follows Fig. 1 and Sections 4.1-4.2 of the paper:

1. every even site n, then every odd site n (Fig. 2 and Section 4.1: sites
   of one parity are uncoupled, so they may be updated in any order or
   simultaneously): propose x_n' = x_n + w * z with all D components moved
   jointly, reject if x_n' leaves the box (Section 4.2), else accept with
   probability min(1, exp(-dA)) (Metropolis rule, Section 3.1);
2. each sampled parameter p_l in ascending l (Fig. 1 step 3): propose
   p_l' = p_l + w_l z, reject outside the box, else compute dA over the whole
   path and accept with the same rule;
3. statistics of the path after the burn-in (Section 4.1).

Readings where the paper is silent or inconsistent:
* colour order: Fig. 1 lists odd first, the text and Fig. 2 even first; even
  first is taken (n = 0 is even);
* proposal law: Gaussian z by default, the U(-1, 1) step of Fig. 1 as an
  option;
* "accept if U(0,1) < P_acc" is taken as: accept iff log u < -dA with
  u = (c + 0.5) 2**-32 from the generator contract (so dA <= 0 always
  accepts); a non-finite dA rejects and is counted;
* the random numbers come from Philox at fixed logical addresses (see
  `philox`) instead of a per-thread Tausworthe stream.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from . import philox as ph
from .action import delta_kinetic, delta_params, delta_site

STATES = 1
PARAMS = 2
GIBBS = 4      # parameters drawn from their exact conditionals (see gibbs.py)
KINETIC = 8    # the Table 1 constants of the gates sampled too (kinetic_moves)

ACC_EVEN, ACC_ODD, ACC_PARAM0, ACC_NONFINITE = 0, 1, 2, 9
N_ACC = 10


@dataclass
class Stats:
    """Shifted moments sum(x - xref), sum((x - xref)^2) over the sweeps
    k >= burn with (k - burn) % stride == 0 (statistics are taken only every
    N_skip-th path update after the initial phase, Section 4.1), the
    parameter vector after every sweep, and acceptance counters.

    With nbatch > 0, batch[b] also sums (x - xref) over the b-th of nbatch
    runs of consecutive samples of one call: the call's i-th sample
    (i = 0 .. ns - 1 of the ns it takes) belongs to batch i * nbatch // ns
    (batch means for the Monte Carlo error of the path means)."""

    M: int
    D: int
    Np: int
    n_sweeps: int
    burn: int = 0
    xref: Optional[np.ndarray] = None
    stride: int = 1
    nbatch: int = 0
    sum: np.ndarray = field(init=False)
    batch: np.ndarray = field(init=False)
    sumsq: np.ndarray = field(init=False)
    ptrace: np.ndarray = field(init=False)
    acc: np.ndarray = field(init=False)
    n_post: int = 0

    def __post_init__(self):
        self.sum = np.zeros((self.M + 1, self.D))
        self.sumsq = np.zeros((self.M + 1, self.D))
        self.batch = np.zeros((self.nbatch, self.M + 1, self.D))
        self.ptrace = np.zeros((self.n_sweeps, self.Np))
        self.acc = np.zeros(N_ACC, dtype=np.int64)
        self.kacc = np.zeros(12, dtype=np.int64)     # accepted moves of each Table 1 constant


@dataclass
class InitPhase:
    """State of the initialization phase of Section 4.2, carried across calls.

    Simulated annealing: the dynamical term of the action carries a
    multiplier beta; the first sweep of the run uses beta0 and beta is
    multiplied by f_beta = (1/beta0)**(1/n_cool) (eq. fbeta) after every
    sweep until it reaches 1 (it is capped there).

    Step sizes: every n_skip-th sweep of the run (k + 1 a multiple of
    n_skip) while k < n_init, every step size is multiplied by
    1 + alpha (N_acc / n_skip - f_acc), N_acc being the accepted changes of
    that path component over the past n_skip sweeps (Section 4.2, the rule
    for Delta_i), and the counts restart.  Reading: the D components of a
    site move jointly with one decision (Fig. 1), so they share N_acc and
    their steps keep the ratios of the base widths: the step of component a
    at site n is w_state[a] * site_scale[n].  Each sampled parameter has
    its own step w_param[l] and count.
    """

    beta0: float
    n_cool: int
    n_init: int
    n_skip: int
    f_acc: float = 0.23
    alpha: float = 0.02
    beta: float = float("nan")                      # beta of the next sweep
    site_scale: Optional[np.ndarray] = None        # (M+1,)
    w_param: Optional[np.ndarray] = None           # (Np,)
    cnt_site: Optional[np.ndarray] = None          # (M+1,) int
    cnt_param: Optional[np.ndarray] = None         # (Np,) int

    def start(self, M, w_param):
        """Fresh state for a run: beta = beta0, unit site scales, the given
        parameter steps, zero counts."""
        self.beta = float(self.beta0)
        self.site_scale = np.ones(M + 1)
        self.w_param = np.array(w_param, dtype=np.float64)
        self.cnt_site = np.zeros(M + 1, dtype=np.int64)
        self.cnt_param = np.zeros(len(self.w_param), dtype=np.int64)
        return self

    @property
    def f_beta(self):
        return (1.0 / self.beta0) ** (1.0 / self.n_cool)


@dataclass
class Debug:
    """What the last sweep proposed and decided (for lockstep comparisons)."""

    xprop: Optional[np.ndarray] = None     # (M+1, D)
    dA: Optional[np.ndarray] = None        # (M+1,), NaN where out of box
    u: Optional[np.ndarray] = None         # (M+1,)
    accept: Optional[np.ndarray] = None    # (M+1,) bool
    pprop: Optional[np.ndarray] = None     # (Np,) proposed value of p_l
    pdA: Optional[np.ndarray] = None       # (Np,)
    pu: Optional[np.ndarray] = None        # (Np,)
    paccept: Optional[np.ndarray] = None   # (Np,) bool
    kprop: Optional[np.ndarray] = None     # (12,) proposed Table 1 constants
    kdA: Optional[np.ndarray] = None
    kaccept: Optional[np.ndarray] = None


def accepts(u, dA):
    """Metropolis decision of Section 3.1: accept with probability
    min(1, exp(-dA)), realised as log u < -dA for u uniform in (0, 1).
    A non-finite dA never accepts."""
    with np.errstate(invalid="ignore"):
        return np.isfinite(dA) & (np.log(u) < -np.asarray(dA, dtype=np.float64))


def site_draws(spec, seed, chain, k, ns):
    """Proposal steps z (len(ns), D) and accept uniforms u for sites ns."""
    ns = np.asarray(ns, dtype=np.int64)
    blk = ph.draw(seed, chain, ns, k, ph.TAG_SITE)
    if spec.proposal == "uniform":
        z = ph.uniforms_pm1(blk)
    else:
        z = ph.normals4(blk)
    acc = ph.draw(seed, chain, ns >> 2, k, ph.TAG_SACC)
    u = ph.uniform_open(acc[np.arange(len(ns)), ns & 3])
    return z[:, :spec.D], u


def param_draw(spec, seed, chain, k, l):
    """Proposal step z and accept uniform u of parameter l (0-based)."""
    b = ph.draw(seed, chain, l, k, ph.TAG_PARAM)[0]
    if spec.proposal == "uniform":
        z = float(ph.uniforms_pm1(b[None, :])[0, 0])
    else:
        z = float(ph.box_muller(b[0], b[1])[0])
    return z, float(ph.uniform_open(b[2]))


def _in_box(x, lo, hi):
    return ((x >= lo) & (x <= hi)).all(axis=-1)


def color_update(spec, X, y, I, p, k, color, w_state, seed, chain, acc=None,
                 order=None, debug: Optional[Debug] = None, site_scale=None, cnt_site=None):
    """Update every site of one parity (in place).

    order=None evaluates the colour at once (legal because same-parity sites
    are uncoupled); otherwise sites are visited one at a time in the given
    permutation of the colour, each against the current path.
    """
    M = X.shape[0] - 1
    ns = np.arange(color, M + 1, 2)
    z, u = site_draws(spec, seed, chain, k, ns)
    w = np.asarray(w_state)[None, :]
    if site_scale is not None:     # per-site steps of the initialization phase
        w = w * site_scale[ns][:, None]
    xprop = X[ns] + w * z
    lo = np.asarray(spec.x_lo)
    hi = np.asarray(spec.x_hi)
    inbox = _in_box(xprop, lo, hi)
    dA = np.full(len(ns), np.nan)
    if order is None:
        if inbox.any():
            dA[inbox] = delta_site(spec, X, y, I, p, ns[inbox], xprop[inbox])
        accept = inbox & accepts(u, dA)
        X[ns[accept]] = xprop[accept]
    else:
        accept = np.zeros(len(ns), dtype=bool)
        for i in order:
            if not inbox[i]:
                continue
            dA[i] = delta_site(spec, X, y, I, p, ns[i:i + 1], xprop[i:i + 1])[0]
            if accepts(u[i], dA[i]):
                accept[i] = True
                X[ns[i]] = xprop[i]
    if acc is not None:
        acc[ACC_EVEN + color] += int(accept.sum())
        acc[ACC_NONFINITE] += int((inbox & ~np.isfinite(dA)).sum())
    if cnt_site is not None:
        cnt_site[ns] += accept
    if debug is not None:
        debug.xprop[ns] = xprop
        debug.dA[ns] = dA
        debug.u[ns] = u
        debug.accept[ns] = accept
    return accept


def param_moves(spec, X, I, p, k, w_param, seed, chain, acc=None,
                debug: Optional[Debug] = None, cnt_param=None):
    """Sequential Metropolis moves of the sampled parameters (in place on p)."""
    lo = np.asarray(spec.p_lo)
    hi = np.asarray(spec.p_hi)
    for l in range(len(p)):
        if not (spec.p_mask >> l) & 1:
            continue
        z, u = param_draw(spec, seed, chain, k, l)
        pp = p.copy()
        pp[l] = p[l] + w_param[l] * z
        dA = np.nan
        ok = False
        if lo[l] <= pp[l] <= hi[l]:
            dA = delta_params(spec, X, I, p, pp)
            ok = bool(accepts(u, dA))
            if not np.isfinite(dA) and acc is not None:
                acc[ACC_NONFINITE] += 1
        if ok:
            p[l] = pp[l]
            if acc is not None:
                acc[ACC_PARAM0 + l] += 1
            if cnt_param is not None:
                cnt_param[l] += 1
        if debug is not None:
            debug.pprop[l] = pp[l]
            debug.pdA[l] = dA
            debug.pu[l] = u
            debug.paccept[l] = ok


def kinetic_moves(spec, X, I, p, k, kin, w_kin, seed, chain, acc=None, debug=None, kacc=None):
    """Sequential Metropolis moves of the sampled Table 1 constants (in place
    on kin, shape (12,) in the order (m, h, n) x (V_a, dV_a, tau0, tau1)).

    Section 5.1 notes that all the constants of the model can be estimated
    with the same method as p.  They enter the gate equations nonlinearly,
    so each move is the paper's direct full pass (Section 4.1): propose
    kin_i + w_i z (Philox KIN block of index i: z from words 0, 1, u from
    word 2), reject outside the box k_lo/k_hi, else accept with the
    Metropolis rule on the change of A summed over the whole path.
    Reading: the constants move after the seven parameters, in the order
    above.  debug, if given, gets kprop/kdA/kaccept (12,)."""
    lo, hi = np.asarray(spec.k_lo), np.asarray(spec.k_hi)
    for i in range(12):
        if not (spec.k_mask >> i) & 1:
            continue
        b = ph.draw(seed, chain, i, k, ph.TAG_KIN)[0]
        z = float(ph.box_muller(b[0], b[1])[0])
        u = float(ph.uniform_open(b[2]))
        prop = kin.copy()
        prop[i] = kin[i] + w_kin[i] * z
        dA, ok = np.nan, False
        if lo[i] <= prop[i] <= hi[i]:
            cur = spec.with_(gates=tuple(tuple(g) for g in kin.reshape(3, 4)))
            dA = delta_kinetic(cur, X, I, p, prop.reshape(3, 4))
            ok = bool(accepts(u, dA))
            if not np.isfinite(dA) and acc is not None:
                acc[ACC_NONFINITE] += 1
        if ok:
            kin[i] = prop[i]
            if kacc is not None:
                kacc[i] += 1
        if debug is not None:
            debug.kprop[i] = prop[i]
            debug.kdA[i] = dA
            debug.kaccept[i] = ok


def run(spec, X, p, y, I, *, seed, chain, sweep0, n_sweeps, w_state, w_param,
        flags=STATES | PARAMS, stats: Optional[Stats] = None,
        debug: Optional[Debug] = None, order_rng: Optional[np.random.Generator] = None,
        init: Optional[InitPhase] = None, kin: Optional[np.ndarray] = None,
        w_kin: Optional[np.ndarray] = None):
    """n_sweeps sweeps k = sweep0 .. sweep0 + n_sweeps - 1, in place on X, p.

    debug, if given, is filled for the last sweep of the call.
    order_rng, if given, visits the sites of each colour in a random order.
    flags & GIBBS draws the parameters from their exact conditionals
    (gibbs.param_gibbs) instead of Metropolis moves.
    init, if given, runs the initialization phase of Section 4.2 (see
    InitPhase; its state is updated in place and w_param is then unused):
    sweep k uses the annealed multiplier init.beta in place of spec.beta.
    kin (12,), if given, holds the Table 1 constants (in/out: they replace
    spec.gates); with flags & KINETIC the constants of spec.k_mask move
    after the parameters (kinetic_moves, steps w_kin).
    """
    from dataclasses import replace

    from .gibbs import param_gibbs
    M = X.shape[0] - 1
    acc = stats.acc if stats is not None else None
    if stats is not None:
        stride = max(stats.stride, 1)
        sampled = [k >= stats.burn and (k - stats.burn) % stride == 0 for k in range(sweep0, sweep0 + n_sweeps)]
        ns, si = sum(sampled), 0
    base_spec = spec
    for i in range(n_sweeps):
        k = sweep0 + i
        if init is not None:
            spec = replace(base_spec, beta=init.beta)
        if kin is not None:
            spec = replace(spec, gates=tuple(tuple(float(v) for v in g) for g in kin.reshape(3, 4)))
        dbg = debug if (debug is not None and i == n_sweeps - 1) else None
        if dbg is not None:
            D = X.shape[1]
            dbg.xprop = np.full((M + 1, D), np.nan)
            dbg.dA = np.full(M + 1, np.nan)
            dbg.u = np.full(M + 1, np.nan)
            dbg.accept = np.zeros(M + 1, dtype=bool)
            dbg.pprop = np.full(len(p), np.nan)
            dbg.pdA = np.full(len(p), np.nan)
            dbg.pu = np.full(len(p), np.nan)
            dbg.paccept = np.zeros(len(p), dtype=bool)
            dbg.kprop = np.full(12, np.nan)
            dbg.kdA = np.full(12, np.nan)
            dbg.kaccept = np.zeros(12, dtype=bool)
        if flags & STATES:
            for color in (0, 1):
                order = None
                if order_rng is not None:
                    order = order_rng.permutation(len(range(color, M + 1, 2)))
                color_update(spec, X, y, I, p, k, color, w_state, seed, chain,
                             acc=acc, order=order, debug=dbg,
                             site_scale=init.site_scale if init is not None else None,
                             cnt_site=init.cnt_site if init is not None else None)
        if flags & PARAMS and flags & GIBBS:
            param_gibbs(spec, X, I, p, k, seed, chain, acc=acc, debug=dbg)
        elif flags & PARAMS:
            param_moves(spec, X, I, p, k, init.w_param if init is not None else w_param, seed, chain,
                        acc=acc, debug=dbg, cnt_param=init.cnt_param if init is not None else None)
        if kin is not None and flags & KINETIC:
            kinetic_moves(spec, X, I, p, k, kin, w_kin, seed, chain, acc=acc, debug=dbg,
                          kacc=stats.kacc if stats is not None else None)
        if init is not None:
            # Section 4.2: beta grows by f_beta after every sweep up to 1; the
            # steps follow the acceptance of the past n_skip sweeps, every
            # n_skip-th sweep of the initialization phase
            init.beta = min(1.0, init.beta * init.f_beta)
            if k < init.n_init and (k + 1) % init.n_skip == 0:
                init.site_scale *= 1.0 + init.alpha * (init.cnt_site / init.n_skip - init.f_acc)
                on = np.array([(base_spec.p_mask >> l) & 1 for l in range(len(p))], dtype=bool)
                upd = 1.0 + init.alpha * (init.cnt_param / init.n_skip - init.f_acc)
                init.w_param[on] *= upd[on]
                init.cnt_site[:] = 0
                init.cnt_param[:] = 0
        if stats is not None:
            stats.ptrace[i] = p
            if sampled[i]:
                d = X - (stats.xref if stats.xref is not None else 0.0)
                stats.sum += d
                stats.sumsq += d * d
                stats.n_post += 1
                if stats.nbatch > 0:
                    stats.batch[si * stats.nbatch // ns] += d
                si += 1
    return X, p
