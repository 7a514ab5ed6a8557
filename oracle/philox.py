"""Philox4x32-10 and the sampler's random-number contract (oracle copy).

Philox4x32-10 is the counter-based generator of Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3" (SC'11): ten rounds of a
multiply/xor bijection of a 128-bit counter under a 64-bit key, with a Weyl
increment of the key between rounds.  It replaces the paper's per-thread
Hybrid Tausworthe generator (Section 4.2), so that every random number has a
fixed logical address independent of how the work is split over threads.

Contract (shared with the HIP library by specification only):
  key      = (seed & 0xffffffff, (seed >> 32) ^ chain)
  counter  = (idx, sweep & 0xffffffff, (tag << 24) | ((sweep >> 32) & 0xffffff), blk)
  tags     SITE   idx = n       4 words -> 4 normals (or 4 uniforms) for site n
           SACC   idx = n >> 2  word n & 3 -> accept uniform of site n
           PARAM  idx = l       words 0,1 -> normal (cos branch) / word 0 uniform;
                                word 2 -> accept uniform of parameter l (0-based)
           MOM    idx = n       4 normals: momentum of site n (HMC)
           PMOM   idx = 0       blk 0 -> params 0..3, blk 1 -> params 4..6 (HMC)
           HACC   idx = 0       word 0 -> HMC accept uniform
  uniform  u = (c + 0.5) * 2**-32 in (0, 1)  (exact in FP64)
  normal   Box-Muller on a word pair (a, b): u_a = (a + 0.5) 2**-32,
           u_b = b 2**-32, r = sqrt(-2 ln u_a), z = (r cos 2 pi u_b, r sin 2 pi u_b)
  box-unif z = 2 u - 1 in (-1, 1)  (the U(-1, 1) step of Fig. 1, step 1a)
"""

from __future__ import annotations

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)

TAG_SITE = 1
TAG_SACC = 2
TAG_PARAM = 3
TAG_MOM = 4
TAG_PMOM = 5
TAG_HACC = 6
TAG_KIN = 7      # moves of the Table 1 kinetic constants

TWO_M32 = 2.0 ** -32


def philox4x32_10(ctr, key) -> np.ndarray:
    """Ten Philox rounds.  ctr: (N, 4) integers < 2**32; key: (2,) or (N, 2).

    Round: with (hi0, lo0) = M0 * c0 and (hi1, lo1) = M1 * c2 as 64-bit
    products, the new counter is (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0);
    the key advances by (W0, W1) between rounds.  Returns (N, 4) uint32.
    """
    c = np.atleast_2d(np.asarray(ctr, dtype=np.uint64)) & _MASK
    k = np.asarray(key, dtype=np.uint64) & _MASK
    if k.ndim == 1:
        k = np.broadcast_to(k, (c.shape[0], 2))
    c0, c1, c2, c3 = c[:, 0].copy(), c[:, 1].copy(), c[:, 2].copy(), c[:, 3].copy()
    k0, k1 = k[:, 0].copy(), k[:, 1].copy()
    m0 = np.uint64(M0)
    m1 = np.uint64(M1)
    for r in range(10):
        if r:
            k0 = (k0 + np.uint64(W0)) & _MASK
            k1 = (k1 + np.uint64(W1)) & _MASK
        p0 = m0 * c0            # < 2**64: exact in uint64
        p1 = m1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return np.stack([c0, c1, c2, c3], axis=1).astype(np.uint32)


def make_key(seed: int, chain: int) -> np.ndarray:
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return np.array([seed & 0xFFFFFFFF, ((seed >> 32) ^ int(chain)) & 0xFFFFFFFF], dtype=np.uint64)


def make_ctr(idx, sweep: int, tag: int, blk=0) -> np.ndarray:
    idx = np.atleast_1d(np.asarray(idx, dtype=np.uint64))
    sweep = int(sweep)
    c = np.empty((idx.shape[0], 4), dtype=np.uint64)
    c[:, 0] = idx & _MASK
    c[:, 1] = sweep & 0xFFFFFFFF
    c[:, 2] = ((tag & 0xFF) << 24) | ((sweep >> 32) & 0xFFFFFF)
    c[:, 3] = np.asarray(blk, dtype=np.uint64)
    return c


def draw(seed: int, chain: int, idx, sweep: int, tag: int, blk=0) -> np.ndarray:
    """Philox block(s) at the contract's address: (N, 4) uint32."""
    return philox4x32_10(make_ctr(idx, sweep, tag, blk), make_key(seed, chain))


def uniform_open(c) -> np.ndarray:
    """u = (c + 0.5) 2**-32, strictly inside (0, 1); exact in FP64."""
    return (np.asarray(c, dtype=np.float64) + 0.5) * TWO_M32


def box_muller(a, b):
    """Two standard normals from two words: (r cos 2 pi u_b, r sin 2 pi u_b)."""
    ua = uniform_open(a)
    ub = np.asarray(b, dtype=np.float64) * TWO_M32
    r = np.sqrt(-2.0 * np.log(ua))
    ang = 2.0 * np.pi * ub
    return r * np.cos(ang), r * np.sin(ang)


def normals4(block: np.ndarray) -> np.ndarray:
    """Four normals per block from word pairs (0, 1) and (2, 3): (N, 4)."""
    z0, z1 = box_muller(block[:, 0], block[:, 1])
    z2, z3 = box_muller(block[:, 2], block[:, 3])
    return np.stack([z0, z1, z2, z3], axis=1)


def uniforms_pm1(block: np.ndarray) -> np.ndarray:
    """Four U(-1, 1) draws per block: 2 u - 1 with u = (c + 0.5) 2**-32."""
    return 2.0 * uniform_open(block) - 1.0
