"""Rademacher probe vectors from Philox4x64-10.  Test infrastructure only.

The paper draws probe entries from {-1, +1} with probability 1/2 (Section 2,
the Hutchinson estimator; Alg 2 and Alg 3, "sample sketching matrix S") but
fixes no generator.  Both the oracle and the GPU library implement the
counter-based Philox4x64 generator with 10 rounds, from its published
definition (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
1, 2, 3", SC'11):

* state: a 4-word counter (c0, c1, c2, c3) and a 2-word key (k0, k1), 64-bit;
* one round: multiply c0 by 0xD2E7470EE14C6C93 and c2 by 0xCA5A826395121157
  into 128-bit products (hi, lo); the new counter is
  (hi(c2 product) ^ c1 ^ k0, lo(c2 product), hi(c0 product) ^ c3 ^ k1,
  lo(c0 product));
* between rounds the key is advanced by the Weyl constants
  (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B).

Probe layout (the only convention both sides share): probe column p, matrix
row i takes the block at counter (i // 256, p, 0, 0) under key (seed, 0); the
bit is bit (i % 64) of output word (i // 64) % 4; a set bit gives -1, a clear
bit +1.  The sketch S holds columns 0..s-1 and the residual probes G columns
s..s+r-1.
"""
from __future__ import annotations

import numpy as np

_MASK = (1 << 64) - 1
_M0 = 0xD2E7470EE14C6C93
_M1 = 0xCA5A826395121157
_W0 = 0x9E3779B97F4A7C15
_W1 = 0xBB67AE8584CAA73B
_ROUNDS = 10


def philox4x64_10(ctr, key):
    """One Philox4x64-10 block with Python integers (exact 128-bit products)."""
    c0, c1, c2, c3 = (int(x) & _MASK for x in ctr)
    k0, k1 = (int(x) & _MASK for x in key)
    for rnd in range(_ROUNDS):
        if rnd > 0:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * c0
        p1 = _M1 * c2
        c0, c1, c2, c3 = ((p1 >> 64) ^ c1 ^ k0, p1 & _MASK,
                          (p0 >> 64) ^ c3 ^ k1, p0 & _MASK)
    return (c0, c1, c2, c3)


def _mulhilo64(a: np.ndarray, b: int):
    """128-bit product of uint64 arrays by a constant, as (hi, lo) uint64,
    from 32-bit limbs (schoolbook multiplication)."""
    m32 = np.uint64(0xFFFFFFFF)
    s32 = np.uint64(32)
    b = np.uint64(b)
    a_lo, a_hi = a & m32, a >> s32
    b_lo, b_hi = b & m32, b >> s32
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> s32) + (lh & m32) + (hl & m32)
    hi = hh + (lh >> s32) + (hl >> s32) + (mid >> s32)
    lo = a * b  # wraps modulo 2^64
    return hi, lo


def philox4x64_10_np(c0, c1, c2, c3, k0: int, k1: int):
    """Vectorised Philox4x64-10 over arrays of counters (uint64), one key."""
    c0 = np.asarray(c0, dtype=np.uint64).copy()
    c1 = np.asarray(c1, dtype=np.uint64).copy()
    c2 = np.asarray(c2, dtype=np.uint64).copy()
    c3 = np.asarray(c3, dtype=np.uint64).copy()
    k0 = int(k0) & _MASK
    k1 = int(k1) & _MASK
    with np.errstate(over="ignore"):
        for rnd in range(_ROUNDS):
            if rnd > 0:
                k0 = (k0 + _W0) & _MASK
                k1 = (k1 + _W1) & _MASK
            hi0, lo0 = _mulhilo64(c0, _M0)
            hi1, lo1 = _mulhilo64(c2, _M1)
            c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1,
                              hi0 ^ c3 ^ np.uint64(k1), lo0)
    return c0, c1, c2, c3


def rademacher(seed: int, n: int, col_begin: int, col_end: int) -> np.ndarray:
    """Probe columns col_begin..col_end-1 as an (n, ncols) float64 array of +-1."""
    ncols = col_end - col_begin
    out = np.empty((n, ncols), dtype=np.float64)
    if n == 0 or ncols == 0:
        return out
    nblk = (n + 255) // 256
    rows = np.arange(n, dtype=np.int64)
    blk = rows // 256
    word = (rows // 64) % 4
    bit = (rows % 64).astype(np.uint64)
    for j in range(ncols):
        p = col_begin + j
        b = np.arange(nblk, dtype=np.uint64)
        w = philox4x64_10_np(b, np.full(nblk, p, dtype=np.uint64),
                             np.zeros(nblk, dtype=np.uint64),
                             np.zeros(nblk, dtype=np.uint64), seed, 0)
        words = np.stack(w, axis=1)  # (nblk, 4)
        bits = (words[blk, word] >> bit) & np.uint64(1)
        out[:, j] = np.where(bits == 1, -1.0, 1.0)
    return out


# ---------------------------------------------------------------------------
# Gaussian probes (the normal alternative the paper allows for the sketch and
# probe vectors, Section 2).  Box-Muller transform (Box & Muller, Ann. Math.
# Stat. 1958) of Philox4x64-10 words: rows 4b..4b+3 of probe column p take the
# block at counter (b, p, 1, 0) under key (seed, 0) - the third counter word
# 1 keeps this stream apart from the Rademacher one.  Words (w0, w1) feed rows
# 4b, 4b+1 and (w2, w3) rows 4b+2, 4b+3; for a pair (wa, wb):
#   u1 = ((wa >> 11) + 1) / 2^53 in (0, 1],  u2 = (wb >> 11) / 2^53 in [0, 1),
#   rho = sqrt(-2 log u1),  even row rho cos(2 pi u2),  odd row rho sin(2 pi u2).
# ---------------------------------------------------------------------------
def gaussian(seed: int, n: int, col_begin: int, col_end: int) -> np.ndarray:
    """Probe columns col_begin..col_end-1 as an (n, ncols) float64 array of N(0, 1) draws."""
    ncols = col_end - col_begin
    out = np.empty((n, ncols), dtype=np.float64)
    if n == 0 or ncols == 0:
        return out
    nblk = (n + 3) // 4
    b = np.arange(nblk, dtype=np.uint64)
    two_pi = 2.0 * np.pi
    scale = 2.0 ** -53
    for j in range(ncols):
        p = col_begin + j
        w = philox4x64_10_np(b, np.full(nblk, p, dtype=np.uint64),
                             np.ones(nblk, dtype=np.uint64),
                             np.zeros(nblk, dtype=np.uint64), seed, 0)
        col = np.empty(4 * nblk)
        for pair in range(2):
            wa, wb = w[2 * pair], w[2 * pair + 1]
            u1 = ((wa >> np.uint64(11)).astype(np.float64) + 1.0) * scale
            u2 = (wb >> np.uint64(11)).astype(np.float64) * scale
            rho = np.sqrt(-2.0 * np.log(u1))
            col[2 * pair::4] = rho * np.cos(two_pi * u2)
            col[2 * pair + 1::4] = rho * np.sin(two_pi * u2)
        out[:, j] = col[:n]
    return out


PROBE_RADEMACHER = 0
PROBE_GAUSSIAN = 1


def probes(seed: int, n: int, col_begin: int, col_end: int, dist: int = PROBE_RADEMACHER) -> np.ndarray:
    """Probe columns of the given distribution (Rademacher or Gaussian)."""
    if dist == PROBE_RADEMACHER:
        return rademacher(seed, n, col_begin, col_end)
    if dist == PROBE_GAUSSIAN:
        return gaussian(seed, n, col_begin, col_end)
    raise ValueError(f"unknown probe distribution {dist}")
