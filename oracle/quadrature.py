"""Reductions of the small projected matrices.  Test infrastructure only.

* Gauss quadrature (Section 3.1, eq. gauss_quadrature): for a unit start
  vector v, v^T f(Q) v is approximated by e1^T f(T_m) e1 =
  sum_k tau_k^2 f(theta_k), where (theta_k, u_k) are the eigenpairs of the
  Lanczos tridiagonal T_m and tau_k = e1^T u_k (the paper's printed
  tau_k^2 = [e1^T u_k] drops the square; the rule needs it).  f = log here;
  a non-positive Ritz value means the operator is not SPD.
* The OSLQ tridiagonal is read off the windowed recurrence: alpha_t = h_{t,t},
  beta_t = h_{t+1,t}; entries above the first superdiagonal (zero in exact
  arithmetic for symmetric Q) are discarded, giving a symmetric T.
* log(H_m) e1 for OSA-IOP (Alg 1): the principal matrix logarithm of the
  Hessenberg matrix, here SciPy's logm (inverse scaling and squaring over a
  Schur form), first column taken.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg


class NotSPDError(ArithmeticError):
    pass


def tridiag_from_hessenberg(h: np.ndarray):
    """(alpha, beta): diagonal and first subdiagonal of H."""
    m = h.shape[0]
    alpha = np.array([h[t, t] for t in range(m)], dtype=np.float64)
    beta = np.array([h[t + 1, t] for t in range(m - 1)], dtype=np.float64)
    return alpha, beta


def gauss_quadrature_log(alpha, beta) -> float:
    """sum_k tau_k^2 log(theta_k) for T = tridiag(beta, alpha, beta)."""
    alpha = np.asarray(alpha, dtype=np.float64)
    beta = np.asarray(beta, dtype=np.float64)
    m = alpha.size
    t = np.diag(alpha)
    if m > 1:
        t += np.diag(beta, 1) + np.diag(beta, -1)
    theta, u = np.linalg.eigh(t)
    if np.any(theta <= 0.0):
        raise NotSPDError(f"non-positive Ritz value {theta.min()!r}")
    tau2 = u[0, :] ** 2
    return float(sum(float(w) * math.log(float(x)) for w, x in zip(tau2, theta)))


def log_hessenberg_e1(h: np.ndarray) -> np.ndarray:
    """First column of the principal logarithm of H."""
    lh = scipy.linalg.logm(np.asarray(h, dtype=np.float64))
    if np.iscomplexobj(lh):
        scale = max(1.0, float(np.max(np.abs(lh.real))))
        if float(np.max(np.abs(lh.imag))) > 1e-8 * scale:
            raise NotSPDError("log(H) is not real: H has eigenvalues off the positive axis")
        lh = lh.real
    return np.ascontiguousarray(lh[:, 0], dtype=np.float64)


def adaptive_dimension(alpha, beta, m_eff: int, broke: bool, m_max: int, every: int,
                       rtol: float) -> int:
    """Krylov dimension at which a run stops under the adaptive rule.

    The paper only names adaptive control of the Krylov dimension (Sections 1
    and 5, with the stop on h < tol of Alg 1); the reading used here: at
    every multiple t of `every` with t < m_max, a run that has not stopped
    forms its Gauss quadrature value K_t on its leading t x t tridiagonal and
    stops at dimension t once |K_t - K_{t - every}| <= rtol |K_t| (the first
    check only records K).  A run that broke down at dimension t is not
    checked there.  rtol <= 0 disables the rule.
    """
    if rtol <= 0.0:
        return m_eff
    prev = None
    t = every
    while t < m_max and t <= m_eff:
        if broke and t == m_eff:
            break
        k_t = gauss_quadrature_log(alpha[:t], beta[:t - 1])
        if prev is not None and abs(k_t - prev) <= rtol * abs(k_t):
            return t
        prev = k_t
        t += every
    return m_eff
