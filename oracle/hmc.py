"""Hybrid Monte Carlo proposal on the path action (oracle, FP64).

The paper names Hybrid Monte Carlo among the methods that sample
exp(-A) (Section 3) and derivative-based proposals as a way to converge in
fewer iterations (Section 3.1).  One proposal, on the coordinates
q = (X, sampled p), with a diagonal mass m per state component and per
parameter:

  r ~ N(0, m)                      (Philox MOM / PMOM addresses)
  H = A(q) + 1/2 sum r^2 / m
  L leapfrog steps of size e:  r -= e/2 dA/dq;  q += e r / m;  r -= e/2 dA/dq
  accept iff log u < -(H_L - H_0)   (u from the HACC address)

Box walls: a coordinate that a drift carries across a wall of its box is
reflected back into the box and its momentum negated (the standard handling
of constraints in HMC: Neal, "MCMC using Hamiltonian dynamics", 2011,
Section 5.1); the map stays reversible and volume preserving, so the target
(exp(-A) on the box) is unchanged.  One reflection per drift: a coordinate
still outside after it (a drift longer than the box) makes the trajectory
invalid, and an invalid trajectory is rejected.  Unsampled parameters keep
zero momentum and never move.
"""

from __future__ import annotations

import numpy as np

from . import philox as ph
from .action import action, grad


def momenta(spec, seed, chain, k, M, minv_state, minv_param):
    D = spec.D
    ns = np.arange(M + 1)
    z = ph.normals4(ph.draw(seed, chain, ns, k, ph.TAG_MOM))[:, :D]
    r = z / np.sqrt(np.asarray(minv_state))[None, :]
    zp = np.concatenate([ph.normals4(ph.draw(seed, chain, 0, k, ph.TAG_PMOM, blk=b))[0] for b in (0, 1)])
    Np = len(minv_param)
    mask = np.array([(spec.p_mask >> l) & 1 for l in range(Np)], dtype=bool)
    rp = np.where(mask, zp[:Np] / np.sqrt(np.asarray(minv_param)), 0.0)
    return r, rp, mask


def kinetic(r, rp, minv_state, minv_param):
    return 0.5 * float((r * r * np.asarray(minv_state)[None, :]).sum()) + \
        0.5 * float((rp * rp * np.asarray(minv_param)).sum())


def reflect(q, r, lo, hi):
    """One reflection at the box walls: returns (q', r', n_reflected, inside)."""
    below = q < lo
    above = q > hi
    q = np.where(below, 2.0 * lo - q, np.where(above, 2.0 * hi - q, q))
    r = np.where(below | above, -r, r)
    inside = bool(((q >= lo) & (q <= hi)).all())
    return q, r, int((below | above).sum()), inside


def leapfrog(spec, X, p, y, I, r, rp, mask, e, L, minv_state, minv_param, count=None):
    """L leapfrog steps from (X, p, r, rp) with reflection at the box walls;
    returns the end point and whether the trajectory stayed valid (every
    drift ended inside the box after at most one reflection).  `count`, a
    one-element list, receives the number of reflections."""
    q = X.copy()
    qp = p.copy()
    r = r.copy()
    rp = rp.copy()
    lo, hi = np.asarray(spec.x_lo), np.asarray(spec.x_hi)
    plo, phi = np.asarray(spec.p_lo), np.asarray(spec.p_hi)
    ms = np.asarray(minv_state)[None, :]
    mp_ = np.asarray(minv_param)
    g, gp = grad(spec, q, y, I, qp)
    inside = True
    for _ in range(L):
        r -= 0.5 * e * g
        rp -= 0.5 * e * np.where(mask, gp, 0.0)
        q += e * ms * r
        qp += e * mp_ * rp
        q, r, n1, ok1 = reflect(q, r, lo[None, :], hi[None, :])
        qs, rs, n2, ok2 = reflect(qp[mask], rp[mask], plo[mask], phi[mask])
        qp[mask] = qs
        rp[mask] = rs
        inside = inside and ok1 and ok2
        if count is not None:
            count[0] += n1 + n2
        g, gp = grad(spec, q, y, I, qp)
        r -= 0.5 * e * g
        rp -= 0.5 * e * np.where(mask, gp, 0.0)
    return q, qp, r, rp, inside


def hmc_proposal(spec, X, p, y, I, *, seed, chain, k, e, L, minv_state, minv_param):
    """One HMC proposal; returns (X', p', accepted, dH)."""
    M = X.shape[0] - 1
    r, rp, mask = momenta(spec, seed, chain, k, M, minv_state, minv_param)
    H0 = action(spec, X, y, I, p)[0] + kinetic(r, rp, minv_state, minv_param)
    q, qp, r1, rp1, inside = leapfrog(spec, X, p, y, I, r, rp, mask, e, L, minv_state, minv_param)
    dH = np.nan
    if inside:
        H1 = action(spec, q, y, I, qp)[0] + kinetic(r1, rp1, minv_state, minv_param)
        dH = H1 - H0
    u = float(ph.uniform_open(ph.draw(seed, chain, 0, k, ph.TAG_HACC)[0, 0]))
    ok = bool(inside and np.isfinite(dH) and np.log(u) < -dH)
    if ok:
        return q, qp, True, dH
    return X.copy(), p.copy(), False, dH
