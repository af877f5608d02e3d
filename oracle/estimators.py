"""OSLQ (Alg 3), OSA-IOP (Alg 2 with Alg 1) and SLQ.  Test infrastructure only.

Both estimators split tr(L_c), L_c = log(Q) - c I, Hutch++-style (Sections
2.2 and 3.3): a sketch S (n x s Rademacher) gives an orthonormal basis A of
range(Y); the subspace part tr(A^T L_c A) is computed run by run and the
residual part is a Hutchinson average over u_j = (I - A A^T) g_j with r
further Rademacher probes; log det Q = n c + tr_sketch + tr_resid.

Readings of the paper used here (each also listed in the design notes):
* split sizes: s sketch columns and r = n_probes - s residual probes, residual
  weight 1/r (the paper's m_vec/3 and 3/m_vec when r = s = m_vec/3);
* the residual update of Alg 3 applies the weight once to the finished sum
  (the printed listing multiplies inside the loop), and its f(theta_k) means
  the residual run's own Ritz values;
* QR convention: the Q-factor with a positive diagonal of R; a sketch image
  that is numerically rank-deficient (the paper does not say what orth()
  returns then) keeps, in column order, the columns whose part orthogonal to
  the columns kept before them exceeds RANK_RTOL of their norm, and the
  basis is the Q-factor of those columns; a dropped column leaves a zero
  column of the basis, whose run is skipped (quadratic form 0, like a
  residual probe that projects to zero);
* OSLQ's "Lanczos" is the windowed recurrence of Alg 1 (window k, MGS order)
  and T keeps only the diagonal and first subdiagonal of H;
* OSA-IOP's sketch line "Y = log(L) S" is read as Y = L_c S, each column from
  Alg 1: y = ||v|| V_m log(H_m) e1 + (log(gamma) - c) v;
* a residual probe that projects to exactly zero contributes zero.

Summation order: sketch terms in column order, residual terms in probe order,
then n c is added to their sum.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np
import scipy.sparse as sp

from .krylov import windowed_arnoldi
from .philox import PROBE_RADEMACHER, probes
from .quadrature import (NotSPDError, adaptive_dimension, gauss_quadrature_log,
                         log_hessenberg_e1, tridiag_from_hessenberg)
from .spectral import osa_iop_shift, oslq_scaling, spectral_interval

DEFAULT_TOL = 1e-10
RANK_RTOL = 1e-6    # relative residual at or below which a sketch column is dependent


@dataclasses.dataclass
class OracleResult:
    logdet: float
    tr_sketch: float
    tr_resid: float
    shift_c: float
    lambda_lo: float
    lambda_hi: float
    scale: float                 # OSLQ: alpha (J = Q/alpha); OSA-IOP: gamma
    probe_K: List[float]         # per run: estimate of x^T L_c x / ||x||^2
    probe_norm2: List[float]     # per run: ||x||^2 of its start vector
    probe_steps: List[int]       # per run: m_eff
    probe_alpha: List[np.ndarray] = dataclasses.field(default_factory=list)
    probe_beta: List[np.ndarray] = dataclasses.field(default_factory=list)
    sketch_basis: Optional[np.ndarray] = None


def _as_scipy(a) -> sp.csr_matrix:
    return sp.csr_matrix((np.asarray(a.values, dtype=np.float64),
                          np.asarray(a.col_idx), np.asarray(a.row_ptr)),
                         shape=(a.n, a.n))


def _orth(y: np.ndarray) -> np.ndarray:
    """Orthonormal basis of range(Y) (the "orthonormal basis via QR" of Alg 2
    and Alg 3), one column per column of Y.

    Columns are taken in order; column j is kept when the part of y_j
    orthogonal to the columns kept before it (Gram-Schmidt applied twice)
    has norm above RANK_RTOL * ||y_j||.  The kept columns' basis is the
    Q-factor of their QR factorisation with diag(R) > 0; a dropped column
    gives a zero column.  For a Y of full column rank this is the Q-factor
    of Y itself."""
    n, s = y.shape
    out = np.zeros_like(y)
    kept = []
    basis = np.zeros((n, 0))
    for j in range(s):
        v = y[:, j]
        nv = float(np.linalg.norm(v))
        w = v - basis @ (basis.T @ v)
        w = w - basis @ (basis.T @ w)
        nw = float(np.linalg.norm(w))
        if nv > 0.0 and nw > RANK_RTOL * nv:
            kept.append(j)
            basis = np.column_stack([basis, w / nw])
    if kept:
        q, r = np.linalg.qr(y[:, kept], mode="reduced")
        d = np.sign(np.diag(r))
        d[d == 0] = 1.0
        out[:, kept] = q * d[None, :]
    return out


def _split(n_probes: int, sketch_rank: int, n: int, m: int, window: int):
    s = int(sketch_rank)
    r = int(n_probes) - s
    if s < 0 or r < 1 or s > n or m < 1 or window < 1:
        raise ValueError(f"bad parameters n_probes={n_probes} sketch_rank={s} "
                         f"krylov_steps={m} iop_window={window} (n={n})")
    return s, r


def oslq(a, n_probes: int, sketch_rank: int, krylov_steps: int, iop_window: int,
         seed: int, tol: float = DEFAULT_TOL, lo_hint: float = 0.0,
         hi_hint: float = 0.0, keep_basis: bool = False,
         dist: int = PROBE_RADEMACHER, adapt_tol: float = 0.0,
         adapt_every: int = 5) -> OracleResult:
    """Alg 3: Hutch++ with the subspace from orth(J S) and Gauss-Lanczos
    quadrature for every quadratic form of log J (optionally with the adaptive
    Krylov dimension of quadrature.adaptive_dimension)."""
    n = a.n
    s, r = _split(n_probes, sketch_rank, n, krylov_steps, iop_window)
    q = _as_scipy(a)
    lo, hi = spectral_interval(a, lo_hint, hi_hint)
    alpha, c = oslq_scaling(lo, hi)

    def apply_j(x):
        return (q @ x) / alpha

    def quad(x):
        h, beta0, _, m_eff, broke = windowed_arnoldi(apply_j, x, krylov_steps, iop_window, tol)
        al, be = tridiag_from_hessenberg(h)
        m_stop = adaptive_dimension(al, be, m_eff, broke, krylov_steps, adapt_every, adapt_tol)
        al, be = al[:m_stop], be[:max(m_stop - 1, 0)]
        return gauss_quadrature_log(al, be), m_stop, al, be

    sk = probes(seed, n, 0, s, dist)
    y = (q @ sk) / alpha if s > 0 else np.zeros((n, 0))
    basis = _orth(y)

    ks, norms, steps, alphas, betas = [], [], [], [], []
    tr_sketch = 0.0
    for i in range(s):
        qi = basis[:, i]
        if not np.any(qi):  # a column dropped by orth(): no run
            ks.append(0.0); norms.append(0.0); steps.append(0)
            alphas.append(np.zeros(0)); betas.append(np.zeros(0))
            continue
        kval, m_eff, al, be = quad(qi)
        tr_sketch += kval
        ks.append(kval); norms.append(float(qi @ qi)); steps.append(m_eff)
        alphas.append(al); betas.append(be)

    g = probes(seed, n, s, s + r, dist)
    acc = 0.0
    for j in range(r):
        u = g[:, j] - basis @ (basis.T @ g[:, j]) if s > 0 else g[:, j].copy()
        nu2 = float(u @ u)
        if nu2 == 0.0:
            ks.append(0.0); norms.append(0.0); steps.append(0)
            alphas.append(np.zeros(0)); betas.append(np.zeros(0))
            continue
        kval, m_eff, al, be = quad(u / math.sqrt(nu2))
        acc += nu2 * kval
        ks.append(kval); norms.append(nu2); steps.append(m_eff)
        alphas.append(al); betas.append(be)
    tr_resid = acc / r
    logdet = n * c + (tr_sketch + tr_resid)
    return OracleResult(logdet, tr_sketch, tr_resid, c, lo, hi, alpha, ks, norms,
                        steps, alphas, betas, basis if keep_basis else None)


def slq(a, n_probes: int, krylov_steps: int, iop_window: int, seed: int,
        tol: float = DEFAULT_TOL, lo_hint: float = 0.0, hi_hint: float = 0.0,
        dist: int = PROBE_RADEMACHER, adapt_tol: float = 0.0, adapt_every: int = 5):
    """Stochastic Lanczos quadrature: the sketch-rank-0 setting of OSLQ."""
    return oslq(a, n_probes, 0, krylov_steps, iop_window, seed, tol, lo_hint, hi_hint,
                dist=dist, adapt_tol=adapt_tol, adapt_every=adapt_every)


def _iop_log_action(q, x, gamma: float, c: float, m: int, window: int, tol: float):
    """Alg 1 on Q~ = Q / gamma, returning (L_c x, m_eff, H, V):
    L_c x = ||x|| V_m log(H_m) e1 + (log(gamma) - c) x."""
    h, beta0, vb, m_eff, _ = windowed_arnoldi(lambda v: (q @ v) / gamma, x, m, window, tol)
    ell = log_hessenberg_e1(h)
    y = np.zeros_like(x)
    for t in range(m_eff):
        y += ell[t] * vb[t]
    y = beta0 * y + (math.log(gamma) - c) * x
    return y, m_eff, h, vb


def osa_iop(a, n_probes: int, sketch_rank: int, krylov_steps: int, iop_window: int,
            seed: int, tol: float = DEFAULT_TOL, lo_hint: float = 0.0,
            hi_hint: float = 0.0, keep_basis: bool = False,
            dist: int = PROBE_RADEMACHER) -> OracleResult:
    """Alg 2: Hutch++ on L_c with every L_c x from Alg 1 (Arnoldi-IOP-LOG)."""
    n = a.n
    s, r = _split(n_probes, sketch_rank, n, krylov_steps, iop_window)
    q = _as_scipy(a)
    lo, hi = spectral_interval(a, lo_hint, hi_hint)
    gamma, c = osa_iop_shift(lo, hi)

    sk = probes(seed, n, 0, s, dist)
    y = np.zeros((n, s))
    for i in range(s):
        y[:, i], _, _, _ = _iop_log_action(q, sk[:, i], gamma, c, krylov_steps, iop_window, tol)
    basis = _orth(y)

    ks, norms, steps, alphas, betas = [], [], [], [], []
    tr_sketch = 0.0
    for i in range(s):
        ai = basis[:, i]
        if not np.any(ai):  # a column dropped by orth(): no run
            ks.append(0.0); norms.append(0.0); steps.append(0)
            alphas.append(np.zeros(0)); betas.append(np.zeros(0))
            continue
        yi, m_eff, h, _ = _iop_log_action(q, ai, gamma, c, krylov_steps, iop_window, tol)
        val = float(ai @ yi)
        nrm = float(ai @ ai)
        tr_sketch += val
        ks.append(val / nrm); norms.append(nrm); steps.append(m_eff)
        al, be = tridiag_from_hessenberg(h)
        alphas.append(al); betas.append(be)

    g = probes(seed, n, s, s + r, dist)
    acc = 0.0
    for j in range(r):
        u = g[:, j] - basis @ (basis.T @ g[:, j]) if s > 0 else g[:, j].copy()
        nu2 = float(u @ u)
        if nu2 == 0.0:
            ks.append(0.0); norms.append(0.0); steps.append(0)
            alphas.append(np.zeros(0)); betas.append(np.zeros(0))
            continue
        yu, m_eff, h, _ = _iop_log_action(q, u, gamma, c, krylov_steps, iop_window, tol)
        val = float(u @ yu)
        acc += val
        ks.append(val / nu2); norms.append(nu2); steps.append(m_eff)
        al, be = tridiag_from_hessenberg(h)
        alphas.append(al); betas.append(be)
    tr_resid = acc / r
    logdet = n * c + (tr_sketch + tr_resid)
    return OracleResult(logdet, tr_sketch, tr_resid, c, lo, hi, gamma, ks, norms,
                        steps, alphas, betas, basis if keep_basis else None)


def dense_logdet(a) -> float:
    """log det of a small matrix from its dense LU (numpy.linalg.slogdet)."""
    dense = _as_scipy(a).toarray()
    sign, val = np.linalg.slogdet(dense)
    if sign <= 0:
        raise NotSPDError("matrix is not positive definite")
    return float(val)


def so_slq(a, n_probes: int, sketch_rank: int, subspace_rank: int, krylov_steps: int,
           iop_window: int, seed: int, tol: float = DEFAULT_TOL, lo_hint: float = 0.0,
           hi_hint: float = 0.0, keep_basis: bool = False,
           dist: int = PROBE_RADEMACHER, adapt_tol: float = 0.0,
           adapt_every: int = 5) -> OracleResult:
    """So-SLQ, the comparator of Section 4 (Han et al.'s subspace construction,
    with the settings the paper gives: a sketch of q = sketch_rank columns and a
    kept rank k = subspace_rank).

    Reading used (the paper describes the method in words only): the sketch is
    Y = log(J) S with J the OSLQ operator (Y = L_c S with OSLQ's shift c, each
    column from Alg 1 on J); the subspace is spanned by the k dominant left
    singular vectors of Y (QR of Y, then the SVD of its R factor); tr(L_c) is
    split as in Hutch++ into the k Gauss-Lanczos quadratic forms on the basis
    vectors and the Hutchinson average over the r = n_probes - q residual
    probes projected off the basis, each also by Gauss-Lanczos quadrature.
    """
    n = a.n
    q_cols = int(sketch_rank)
    k_rank = int(subspace_rank)
    r = int(n_probes) - q_cols
    if q_cols < 1 or k_rank < 1 or k_rank > q_cols or q_cols > n or r < 1 \
            or krylov_steps < 1 or iop_window < 1:
        raise ValueError(f"bad So-SLQ parameters n_probes={n_probes} sketch_rank={q_cols} "
                         f"subspace_rank={k_rank}")
    q = _as_scipy(a)
    lo, hi = spectral_interval(a, lo_hint, hi_hint)
    alpha, c = oslq_scaling(lo, hi)

    def apply_j(x):
        return (q @ x) / alpha

    def quad(x):
        h, beta0, _, m_eff, broke = windowed_arnoldi(apply_j, x, krylov_steps, iop_window, tol)
        al, be = tridiag_from_hessenberg(h)
        m_stop = adaptive_dimension(al, be, m_eff, broke, krylov_steps, adapt_every, adapt_tol)
        al, be = al[:m_stop], be[:max(m_stop - 1, 0)]
        return gauss_quadrature_log(al, be), m_stop, al, be

    # sketch of the traced operator log(J) = L_c, one Alg 1 run per column
    sk = probes(seed, n, 0, q_cols, dist)
    y = np.zeros((n, q_cols))
    for i in range(q_cols):
        y[:, i], _, _, _ = _iop_log_action(q, sk[:, i], alpha, c, krylov_steps, iop_window, tol)
    qy = _orth(y)
    rfac = qy.T @ y
    u_r, sig, _ = np.linalg.svd(rfac)
    basis = qy @ u_r[:, :k_rank]

    ks, norms, steps, alphas, betas = [], [], [], [], []
    tr_sketch = 0.0
    for i in range(k_rank):
        bi = basis[:, i]
        kval, m_eff, al, be = quad(bi / math.sqrt(float(bi @ bi)))
        tr_sketch += kval
        ks.append(kval); norms.append(float(bi @ bi)); steps.append(m_eff)
        alphas.append(al); betas.append(be)

    g = probes(seed, n, q_cols, q_cols + r, dist)
    acc = 0.0
    for j in range(r):
        u = g[:, j] - basis @ (basis.T @ g[:, j])
        nu2 = float(u @ u)
        if nu2 == 0.0:
            ks.append(0.0); norms.append(0.0); steps.append(0)
            alphas.append(np.zeros(0)); betas.append(np.zeros(0))
            continue
        kval, m_eff, al, be = quad(u / math.sqrt(nu2))
        acc += nu2 * kval
        ks.append(kval); norms.append(nu2); steps.append(m_eff)
        alphas.append(al); betas.append(be)
    tr_resid = acc / r
    logdet = n * c + (tr_sketch + tr_resid)
    return OracleResult(logdet, tr_sketch, tr_resid, c, lo, hi, alpha, ks, norms,
                        steps, alphas, betas, basis if keep_basis else None)
