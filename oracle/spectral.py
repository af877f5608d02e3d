"""Spectral interval and the shift/scale rules.  Test infrastructure only.

* Gershgorin interval (Section 2.1): lmin >= min_i (a_ii - sum_{j!=i} |a_ij|),
  lmax <= max_i (a_ii + sum_{j!=i} |a_ij|).  When the lower bound is not
  positive the paper substitutes an unspecified small positive threshold; we
  read that as GERSH_FLOOR_REL * lmax.  A caller-supplied hint (> 0) replaces
  the corresponding bound; a hint is applied before the floor.
* gamma = sqrt(lmin lmax) (Proposition 2.1), the scale of Q~ = Q / gamma.
* The traced operator is made PSD by a constant shift (the definitions of L in
  Section 2.2 and of J in Section 3.2).  Both cases are written here as
  L_c = log(Q) - c I and log det Q = n c + tr(L_c):
    - OSLQ: J = Q / lmax and c = log(lmax) when lmin < 1, else J = Q and
      c = 0 (the paper's output line carries n log(alpha) in both branches,
      which only holds for the first one).
    - OSA-IOP: c = log(lmin) when lmin < 1 (alpha = lmin(Q)), else
      c = log(gamma) (L = log Q~ in the "otherwise" branch).
  The branch tests use the lower bound of the interval because the exact
  smallest eigenvalue is unknown.
"""
from __future__ import annotations

import math

import numpy as np

GERSH_FLOOR_REL = 1e-6


def gershgorin_bounds(a):
    """(lo, hi) Gershgorin bounds of a CSR matrix (n, row_ptr, col_idx, values).

    Row i: centre a_ii, radius sum_{j != i} |a_ij|, both summed in the row's
    stored order."""
    n = a.n
    counts = np.diff(np.asarray(a.row_ptr, dtype=np.int64))
    rows = np.repeat(np.arange(n, dtype=np.int64), counts)
    cols = np.asarray(a.col_idx, dtype=np.int64)
    vals = np.asarray(a.values, dtype=np.float64)
    on = cols == rows
    centre = np.bincount(rows[on], weights=vals[on], minlength=n)
    radius = np.bincount(rows[~on], weights=np.abs(vals[~on]), minlength=n)
    return float(np.min(centre - radius)), float(np.max(centre + radius))


def spectral_interval(a, lo_hint: float = 0.0, hi_hint: float = 0.0):
    """Interval [lo, hi] used by both estimators."""
    lo, hi = gershgorin_bounds(a)
    if hi_hint > 0.0:
        hi = float(hi_hint)
    if lo_hint > 0.0:
        lo = float(lo_hint)
    if lo <= 0.0:
        lo = GERSH_FLOOR_REL * hi
    if not (0.0 < lo <= hi) or not math.isfinite(hi):
        raise ValueError(f"bad spectral interval [{lo}, {hi}]")
    return lo, hi


def oslq_scaling(lo: float, hi: float):
    """(alpha, c): OSLQ runs on J = Q / alpha, and log det Q = n c + tr log J."""
    if lo < 1.0:
        return hi, math.log(hi)
    return 1.0, 0.0


def osa_iop_shift(lo: float, hi: float):
    """(gamma, c): Krylov runs on Q / gamma; traced operator log Q - c I."""
    gamma = math.sqrt(lo * hi)
    c = math.log(lo) if lo < 1.0 else math.log(gamma)
    return gamma, c
