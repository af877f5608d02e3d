"""Pins of the windowed Arnoldi/IOP recurrence (Alg 1) (CPU only)."""
import numpy as np
import pytest

import workloads as W
from oracle import windowed_arnoldi


def _op(q):
    return lambda x: q @ x


@pytest.mark.parametrize("window", [1, 2, 3, 5, 100])
def test_polynomial_exactness(window):
    # Appendix A (eq. poly-commute): ||v|| V_m p(H_m) e1 = p(Q) v for any
    # polynomial of degree <= m-1; it holds for the incomplete (non-orthogonal)
    # basis too, because Q V_m = V_m H_m + h v_{m+1} e_m^T holds by construction.
    n, m = 40, 12
    q = W.random_spd_dense(n, seed=11, lo=0.5, hi=2.0)
    rng = np.random.default_rng(0)
    v = rng.standard_normal(n)
    h, beta0, vb, m_eff, broke = windowed_arnoldi(_op(q), v, m, window, 1e-12)
    assert m_eff == m and not broke
    vm = np.stack(vb, axis=1)
    coeffs = rng.standard_normal(m)  # degree m-1
    e1 = np.zeros(m); e1[0] = 1.0
    lhs = np.zeros(n)
    pw = e1.copy()
    pv = v.copy()
    rhs = np.zeros(n)
    for d in range(m):
        lhs += coeffs[d] * (vm @ pw)
        rhs += coeffs[d] * pv
        pw = h @ pw
        pv = q @ pv
    np.testing.assert_allclose(beta0 * lhs, rhs, rtol=1e-9, atol=1e-9 * np.linalg.norm(rhs))


def test_full_window_is_orthonormal_projection():
    n, m = 30, 10
    q = W.random_spd_dense(n, seed=5)
    v = np.random.default_rng(1).standard_normal(n)
    h, beta0, vb, m_eff, _ = windowed_arnoldi(_op(q), v, m, m, 1e-12)
    vm = np.stack(vb, axis=1)
    np.testing.assert_allclose(vm.T @ vm, np.eye(m), atol=1e-12)
    np.testing.assert_allclose(h, vm.T @ q @ vm, atol=1e-11)
    assert beta0 == pytest.approx(np.linalg.norm(v))


def test_window_two_is_three_term_for_symmetric():
    # for symmetric Q the window-2 recurrence is Lanczos: H is tridiagonal
    # and symmetric up to rounding
    n, m = 50, 15
    q = W.random_spd_dense(n, seed=8, lo=1.0, hi=3.0)
    v = np.random.default_rng(2).standard_normal(n)
    h, _, vb, _, _ = windowed_arnoldi(_op(q), v, m, 2, 1e-12)
    assert np.all(np.triu(h, 2) == 0.0)
    np.testing.assert_allclose(np.diag(h, 1), np.diag(h, -1), rtol=1e-10)
    # each new vector is orthogonal to its two predecessors
    for t in range(2, m):
        assert abs(vb[t] @ vb[t - 1]) < 1e-12 and abs(vb[t] @ vb[t - 2]) < 1e-12


def test_mgs_order_within_window():
    # coefficients are taken on the already-updated w, oldest vector first:
    # reproduce column t by hand for a non-symmetric operator
    n, m, k = 12, 6, 3
    rng = np.random.default_rng(4)
    a = rng.standard_normal((n, n)) + 4 * np.eye(n)
    v = rng.standard_normal(n)
    h, beta0, vb, _, _ = windowed_arnoldi(_op(a), v, m, k, 1e-14)
    t = 4
    w = a @ vb[t]
    for j in (2, 3, 4):
        c = vb[j] @ w
        assert h[j, t] == pytest.approx(c, rel=1e-12, abs=1e-14)
        w = w - c * vb[j]
    assert h[0, t] == 0.0 and h[1, t] == 0.0
    np.testing.assert_allclose(vb[t + 1], w / np.linalg.norm(w), atol=1e-13)


def test_breakdown_on_d_distinct_eigenvalues():
    # a diagonal matrix with d distinct values has a d-dimensional Krylov
    # space: h_{d+1,d} falls below tol and m_eff = d
    d_vals = np.repeat(np.array([0.5, 1.0, 2.0, 3.0]), 5)
    a = W.diag_matrix(d_vals).to_scipy()
    v = np.ones(d_vals.size)
    h, _, _, m_eff, broke = windowed_arnoldi(lambda x: a @ x, v, 10, 10, 1e-10)
    assert broke and m_eff == 4 and h.shape == (4, 4)
    # the Ritz values are then exactly the distinct eigenvalues
    np.testing.assert_allclose(np.sort(np.linalg.eigvals(h).real), [0.5, 1.0, 2.0, 3.0], atol=1e-10)
