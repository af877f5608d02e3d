"""Accuracy of the Gauss quadrature kernels on their own: K = e1^T log(T) e1
for symmetric tridiagonal T (Section 2's Gauss quadrature of the Lanczos
runs), as the estimates compute it (trapezoidal rule on the Stieltjes
integral of log, Golub-Welsch where T leaves the trusted interval).

Inputs are the tridiagonals of FP64 Lanczos runs with full
reorthogonalisation on diagonal operators whose spectra fill [a, b], the
interval the estimate passes to the kernel, plus runs whose Ritz values leave
[a/1000, 1000 b] (the Golub-Welsch path).  References: the oracle's
eigendecomposition rule, and for a subset the same sum in 40-digit
arithmetic (mpmath), which also pins the oracle.  Gate 1e-12 absolute (|K|
is at most a few units here).
"""
import numpy as np
import pytest

import oracle.quadrature as Q

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    from paper_2606_07004_amd import liblogdet
    liblogdet.lib()  # fails loudly when the HIP library is missing
    return liblogdet


@pytest.fixture(scope="module")
def ctx(L):
    c = L.Context(0)
    yield c
    c.close()


def _lanczos_tridiagonal(rng, eigs, m):
    """alpha[m], beta[m] (beta[t] = T[t+1, t]) of m Lanczos steps on diag(eigs)
    from a random start, full reorthogonalisation."""
    n = len(eigs)
    V = np.zeros((n, m + 1))
    v = rng.standard_normal(n)
    V[:, 0] = v / np.linalg.norm(v)
    al, be = np.zeros(m), np.zeros(m)
    for t in range(m):
        w = eigs * V[:, t]
        al[t] = V[:, t] @ w
        for _ in range(2):
            w -= V[:, : t + 1] @ (V[:, : t + 1].T @ w)
        be[t] = np.linalg.norm(w)
        V[:, t + 1] = w / be[t]
    return al, be


def _cases(seed, count, m_max):
    rng = np.random.default_rng(seed)
    al = np.zeros((count, m_max))
    be = np.zeros((count, m_max))
    dims = np.zeros(count, dtype=np.int32)
    for p in range(count):
        a = [1e-3, 0.05, 0.5][p % 3]
        b = a * 10 ** rng.uniform(0.3, 3.3)
        eigs = np.sort(np.concatenate([[a, b], rng.uniform(a, b, 300)]))
        m = int(rng.integers(1, m_max + 1))
        al[p, :m], be[p, :m] = _lanczos_tridiagonal(rng, eigs, m)
        dims[p] = m
    return al, be, dims


def _oracle_K(al, be, dims):
    return np.array([Q.gauss_quadrature_log(al[p, : dims[p]], be[p, : dims[p] - 1])
                     for p in range(len(dims))])


def test_trapezoidal_rule_matches_eigh(L, ctx):
    print("\n[case] k_quad_log on 240 Lanczos tridiagonals, spectra in [a, b]", flush=True)
    al, be, dims = _cases(0, 240, 50)
    worst = 0.0
    for a_run, (lo, hi) in enumerate([(1e-3, None), (0.05, None), (0.5, None)]):
        sel = np.arange(a_run, len(dims), 3)
        a = lo
        # the interval the estimate would pass: the operator's bounds
        b = max(float(np.max(al[sel])) * 4, lo * 2)
        K, need = L.ld_debug_quad_log(ctx.handle, al[sel], be[sel], dims[sel], a, b)
        ref = _oracle_K(al[sel], be[sel], dims[sel])
        assert not need.any()  # every Ritz value inside [a, b]: the trapezoidal rule
        err = np.abs(K - ref)
        worst = max(worst, float(err.max()))
        np.testing.assert_allclose(K, ref, rtol=0, atol=1e-12)
    print(f"  worst |K - K_eigh| = {worst:.2e}", flush=True)


def test_golub_welsch_fallback_matches_eigh(L, ctx):
    print("\n[case] Golub-Welsch fallback: Ritz values below a/1000", flush=True)
    al, be, dims = _cases(1, 60, 40)
    # claim a lower bound 1e4 times above the smallest eigenvalue of each
    # family: the runs that reach it leave the trusted interval
    K, need = L.ld_debug_quad_log(ctx.handle, al, be, dims, 20.0, 2000.0)
    ref = _oracle_K(al, be, dims)
    theta_min = np.array([np.linalg.eigvalsh(np.diag(al[p, : dims[p]]) +
                                             np.diag(be[p, : dims[p] - 1], 1) +
                                             np.diag(be[p, : dims[p] - 1], -1)).min()
                          for p in range(len(dims))])
    np.testing.assert_array_equal(need, (theta_min < 20.0 / 1000).astype(np.int32))
    assert need.sum() >= 10
    np.testing.assert_allclose(K, ref, rtol=0, atol=1e-12)


def test_against_extended_precision(L, ctx):
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 40
    print("\n[case] quadrature kernels and oracle against 40-digit eigensums", flush=True)
    al, be, dims = _cases(2, 12, 24)
    a, b = 1e-3, float(np.max(al)) * 4
    K, need = L.ld_debug_quad_log(ctx.handle, al, be, dims, a, b)
    ref64 = _oracle_K(al, be, dims)
    for p in range(len(dims)):
        m = int(dims[p])
        T = mpmath.matrix(m, m)
        for t in range(m):
            T[t, t] = mpmath.mpf(float(al[p, t]))
            if t + 1 < m:
                T[t + 1, t] = T[t, t + 1] = mpmath.mpf(float(be[p, t]))
        E, U = mpmath.eigsy(T)
        exact = float(mpmath.fsum(U[0, i] ** 2 * mpmath.log(E[i]) for i in range(m)))
        assert abs(ref64[p] - exact) <= 1e-12
        assert abs(K[p] - exact) <= 1e-12
