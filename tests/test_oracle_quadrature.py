"""Pins of the Gauss quadrature and log(H) e1 helpers (CPU only)."""
import math

import numpy as np
import pytest
import scipy.linalg

import oracle as O
import workloads as W
from oracle import (NotSPDError, gauss_quadrature_log, log_hessenberg_e1,
                    tridiag_from_hessenberg, windowed_arnoldi)


@pytest.mark.parametrize("m", [1, 2, 5, 12])
def test_legendre_jacobi_matrix_gives_gauss_legendre(m):
    # The Jacobi matrix of the Legendre weight (alpha = 0,
    # beta_j = j / sqrt(4 j^2 - 1)) has the Gauss-Legendre nodes as
    # eigenvalues and weights 2 tau_k^2.  Probe the oracle's rule with
    # f = log on the shifted matrix T + 3 I: sum tau^2 log(theta + 3) must
    # equal (1/2) sum w_k log(x_k + 3).
    j = np.arange(1, m)
    beta = j / np.sqrt(4.0 * j * j - 1.0)
    alpha = np.zeros(m)
    x, w = np.polynomial.legendre.leggauss(m)
    ref = 0.5 * float(np.sum(w * np.log(x + 3.0)))
    assert gauss_quadrature_log(alpha + 3.0, beta) == pytest.approx(ref, rel=1e-13, abs=1e-14)


def test_quadrature_exact_for_low_degree_polynomials():
    # with m = n Krylov steps the Gauss rule reproduces the spectral measure
    # of the unit start vector, so it is exact for every f, log included:
    # sum tau^2 log(theta) = sum_i (u_i^T v)^2 log(lambda_i).
    n = 14
    q = W.random_spd_dense(n, seed=21, lo=0.2, hi=5.0)
    v = np.random.default_rng(3).standard_normal(n)
    v /= np.linalg.norm(v)
    h, _, _, m_eff, _ = windowed_arnoldi(lambda x: q @ x, v, n, n, 1e-13)
    al, be = tridiag_from_hessenberg(h)
    lam, u = np.linalg.eigh(q)
    exact = float(np.sum((u.T @ v) ** 2 * np.log(lam)))
    assert gauss_quadrature_log(al, be) == pytest.approx(exact, rel=1e-11)


def test_quadrature_moments_match_krylov_moments():
    # moments: e1^T T^p e1 = v^T Q^p v for p <= 2m-1 (full re-orthogonalisation)
    n, m = 60, 6
    q = W.random_spd_dense(n, seed=2, lo=0.5, hi=2.0)
    v = np.random.default_rng(9).standard_normal(n)
    v /= np.linalg.norm(v)
    h, _, _, _, _ = windowed_arnoldi(lambda x: q @ x, v, m, m, 1e-13)
    al, be = tridiag_from_hessenberg(h)
    t = np.diag(al) + np.diag(be, 1) + np.diag(be, -1)
    for p in range(2 * m):
        e1 = np.zeros(m); e1[0] = 1
        lhs = e1 @ np.linalg.matrix_power(t, p) @ e1
        rhs = v @ np.linalg.matrix_power(q, p) @ v
        assert lhs == pytest.approx(rhs, rel=1e-9)
    # and the log rule uses exactly these moments: first-order check via
    # the quadrature of log on a tiny diagonal T
    assert gauss_quadrature_log([2.0], []) == pytest.approx(math.log(2.0))


def test_quadrature_rejects_non_spd():
    with pytest.raises(NotSPDError):
        gauss_quadrature_log([1.0, -0.5], [0.1])


def test_tridiag_from_hessenberg():
    h = np.arange(16.0).reshape(4, 4)
    al, be = tridiag_from_hessenberg(h)
    np.testing.assert_array_equal(al, [0, 5, 10, 15])
    np.testing.assert_array_equal(be, [4, 9, 14])


def test_log_hessenberg_symmetric_case_matches_eigh():
    rng = np.random.default_rng(5)
    m = 9
    al = rng.uniform(0.5, 3.0, m)
    be = rng.uniform(0.05, 0.3, m - 1)
    t = np.diag(al) + np.diag(be, 1) + np.diag(be, -1)
    lam, u = np.linalg.eigh(t)
    ref = u @ (np.log(lam) * u[0, :])
    np.testing.assert_allclose(log_hessenberg_e1(t), ref, rtol=1e-12, atol=1e-13)
    # e1^T log(T) e1 is the Gauss quadrature value
    assert log_hessenberg_e1(t)[0] == pytest.approx(gauss_quadrature_log(al, be), rel=1e-12)


def test_log_hessenberg_nonsymmetric_integral_representation():
    # Independent route: log(H) = int_0^1 (H - I) (t (H - I) + I)^{-1} dt for a
    # matrix with spectrum off the closed negative axis; apply it to e1 with a
    # 80-point Gauss-Legendre rule in t (solves only, no logm).
    rng = np.random.default_rng(6)
    m = 10
    h = np.triu(rng.uniform(-0.2, 0.2, (m, m)), -1)
    h[np.arange(m), np.arange(m)] = rng.uniform(0.5, 2.0, m)
    e1 = np.zeros(m); e1[0] = 1.0
    x, w = np.polynomial.legendre.leggauss(80)
    tt, ww = 0.5 * (x + 1.0), 0.5 * w
    b = (h - np.eye(m)) @ e1
    ref = sum(wk * np.linalg.solve(tk * (h - np.eye(m)) + np.eye(m), b) for tk, wk in zip(tt, ww))
    np.testing.assert_allclose(log_hessenberg_e1(h), ref, rtol=1e-11, atol=1e-12)


def test_log_hessenberg_rejects_negative_spectrum():
    h = np.array([[-1.0, 0.2], [0.3, 2.0]])
    with pytest.raises(NotSPDError):
        log_hessenberg_e1(h)


# ---------------------------------------------------------------------------
# Adaptive Krylov dimension (stop once the quadrature value settles)
# ---------------------------------------------------------------------------
from oracle.quadrature import adaptive_dimension  # noqa: E402


def test_adaptive_dimension_on_decoupled_tridiagonal():
    # beta_5 = 0 decouples T after row 5: e1 sees only the leading 5 x 5 block,
    # so K_t = K_5 for t >= 5.  Checks every 3: t = 3 records, t = 6 differs
    # from K_3, t = 9 equals K_6 -> stop at 9.  A run that broke down at its
    # last dimension is not checked there; rtol 0 never stops.
    rng = np.random.default_rng(3)
    al = rng.uniform(0.2, 0.9, 20)
    be = rng.uniform(0.05, 0.1, 19)
    be[4] = 0.0
    assert adaptive_dimension(al, be, 20, False, 20, 3, 1e-12) == 9
    assert adaptive_dimension(al, be, 9, True, 20, 3, 1e-12) == 9   # not checked at 9
    assert adaptive_dimension(al, be, 20, False, 20, 3, 0.0) == 20
    assert adaptive_dimension(al, be, 20, False, 9, 3, 1e-12) == 20  # t < m_max only


def test_adaptive_rtol_zero_is_the_plain_estimator():
    a = W.lap2d(20, 0.1)
    r0 = O.oslq(a, 12, 4, 30, 2, 1)
    r1 = O.oslq(a, 12, 4, 30, 2, 1, adapt_tol=0.0, adapt_every=4)
    assert r0.logdet == r1.logdet and r0.probe_steps == r1.probe_steps


def test_adaptive_estimate_close_to_converged_one():
    # geometric convergence of Gauss quadrature on a well-conditioned operator:
    # the adaptive estimate is within a few rtol of the full-depth estimate and
    # uses fewer steps; a tighter rtol never uses fewer steps
    a = W.lap2d(30, 0.5)
    full = O.oslq(a, 12, 4, 60, 60, 2)
    steps = []
    for rtol in (1e-3, 1e-6, 1e-9):
        r = O.oslq(a, 12, 4, 60, 60, 2, adapt_tol=rtol, adapt_every=4)
        rel = abs(r.logdet - full.logdet) / abs(full.logdet)
        assert rel <= 10 * rtol
        assert max(r.probe_steps) < 60
        steps.append(sum(r.probe_steps))
    assert steps[0] <= steps[1] <= steps[2]


def test_gauss_quadrature_log_against_extended_precision():
    # the same sum, e1^T log(T) e1 = sum_i u_{1i}^2 log(theta_i), from a
    # 40-digit eigendecomposition: the FP64 rule must agree to 1e-13
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 40
    rng = np.random.default_rng(11)
    for trial in range(8):
        m = int(rng.integers(2, 20))
        d = rng.uniform(0.01, 50.0, m)
        e = rng.uniform(-2.0, 2.0, m - 1)
        t = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
        lam = np.linalg.eigvalsh(t)
        if lam.min() <= 0:
            d = d + (0.05 - lam.min())
        M = mpmath.matrix(m, m)
        for i in range(m):
            M[i, i] = mpmath.mpf(float(d[i]))
            if i + 1 < m:
                M[i + 1, i] = M[i, i + 1] = mpmath.mpf(float(e[i]))
        E, U = mpmath.eigsy(M)
        exact = float(mpmath.fsum(U[0, i] ** 2 * mpmath.log(E[i]) for i in range(m)))
        assert abs(gauss_quadrature_log(d, e) - exact) <= 1e-13 * max(1.0, abs(exact))
