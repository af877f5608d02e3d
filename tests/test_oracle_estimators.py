"""Pins of the OSLQ / OSA-IOP oracle estimators (CPU only).

Each check fixes the oracle to something other than itself: dense
log-determinants (LU), closed-form Laplacian eigenvalues, exact Hutch++
identities when the sketch spans the traced operator, exact scale identities,
unbiasedness over seeds, and an independent dense evaluation of the
quadratic forms.
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle.philox import rademacher


def _full_rank_seed(n, s, start=0):
    for seed in range(start, start + 200):
        if np.linalg.matrix_rank(rademacher(seed, n, 0, s)) == min(n, s):
            return seed
    raise RuntimeError("no full-rank sketch found")


def _dense_logm(q):
    lam, u = np.linalg.eigh(q)
    return (u * np.log(lam)) @ u.T


def test_laplacian_closed_forms_match_dense():
    for n2, sh in ((7, 0.1), (5, 1e-3)):
        a = W.lap2d(n2, sh)
        assert W.lap2d_exact_logdet(n2, sh) == pytest.approx(O.dense_logdet(a), rel=1e-13)
    a = W.lap3d(4, 0.2)
    assert W.lap3d_exact_logdet(4, 0.2) == pytest.approx(O.dense_logdet(a), rel=1e-13)


@pytest.mark.parametrize("method", ["oslq", "osa_iop"])
def test_full_sketch_is_exact(method):
    # s = n: A spans R^n, the residual vanishes, and with m = n full
    # re-orthogonalisation every quadratic form is exact, so the estimate is
    # log det Q itself.
    n = 8
    q = W.random_spd_dense(n, seed=4, lo=0.3, hi=4.0)
    a = W.from_dense(q)
    seed = _full_rank_seed(n, n)
    fn = getattr(O, method)
    res = fn(a, n_probes=n + 1, sketch_rank=n, krylov_steps=n, iop_window=n, seed=seed)
    assert res.logdet == pytest.approx(O.dense_logdet(a), rel=1e-10, abs=1e-10)
    assert abs(res.tr_resid) < 1e-10


def test_osa_iop_exact_when_traced_operator_has_rank_s():
    # Hutch++ exactness: if rank(L_c) <= s the sketch Y = L_c S spans
    # range(L_c); tr(A^T L_c A) = tr(L_c) and every residual form is 0.
    # Q diagonal: 26 entries at the lower bound 0.2 (so L_c = log Q - log 0.2
    # vanishes there) and 4 distinct larger values.
    d = np.concatenate([np.full(26, 0.2), [0.5, 1.3, 2.0, 3.7]])
    a = W.diag_matrix(d)
    s = 4
    seed = None
    for sd in range(200):
        if np.linalg.matrix_rank(rademacher(sd, 30, 0, s)[26:, :]) == s:
            seed = sd
            break
    res = O.osa_iop(a, n_probes=7, sketch_rank=s, krylov_steps=10, iop_window=2, seed=seed)
    assert res.shift_c == pytest.approx(math.log(0.2))
    assert res.logdet == pytest.approx(float(np.sum(np.log(d))), rel=1e-10)
    assert abs(res.tr_resid) < 1e-10


def test_oslq_scale_identity():
    # A = orth(J S) does not depend on the scale alpha, and a unit-vector
    # quadrature of log(Q/alpha) equals that of log Q minus log alpha.  So two
    # upper hints h1, h2 (c_i = log h_i) give
    #   est1 - est2 = (c1 - c2) (n - s - (1/r) sum_j ||u_j||^2).
    a = W.lap2d(12, 0.1)
    s, npr = 6, 16
    r = npr - s
    e1 = O.oslq(a, npr, s, 20, 20, seed=3)
    e2 = O.oslq(a, npr, s, 20, 20, seed=3, hi_hint=11.0)
    assert e1.shift_c == pytest.approx(math.log(8.1)) and e2.shift_c == pytest.approx(math.log(11.0))
    coef = a.n - s - sum(e1.probe_norm2[s:]) / r
    assert e1.logdet - e2.logdet == pytest.approx((e1.shift_c - e2.shift_c) * coef,
                                                  abs=1e-9 * abs(e1.logdet))
    for k1, k2 in zip(e1.probe_K, e2.probe_K):
        assert k1 - k2 == pytest.approx(e2.shift_c - e1.shift_c, abs=1e-10)


def test_osa_iop_gamma_invariance():
    # K_m(Q/gamma, v) = K_m(Q, v) and H(Q/gamma) = H(Q)/gamma, so the
    # log(gamma) term of Alg 1 cancels exactly: with c fixed (c = log lo),
    # changing gamma through the upper hint leaves the estimate unchanged.
    a = W.lap2d(12, 0.1)
    e1 = O.osa_iop(a, 15, 5, 12, 2, seed=1)
    e2 = O.osa_iop(a, 15, 5, 12, 2, seed=1, hi_hint=40.0)
    assert e1.scale != pytest.approx(e2.scale)
    assert e1.shift_c == e2.shift_c
    assert e1.logdet == pytest.approx(e2.logdet, rel=1e-10)


@pytest.mark.parametrize("method", ["oslq", "osa_iop"])
def test_matches_dense_quadratic_forms(method):
    # With m = n and full re-orthogonalisation every Krylov quadratic form is
    # exact, so the estimate must equal the Hutch++ split evaluated with the
    # dense matrix logarithm (eigendecomposition), on the same basis A and
    # the same residual probes.  (The matrix has a simple spectrum so that
    # m = n steps do not run past an exhausted Krylov space.)
    a = W.from_dense(W.random_spd_dense(24, seed=31, lo=0.3, hi=5.0))
    n = a.n
    s, npr = 5, 12
    r = npr - s
    q = a.to_dense()
    res = getattr(O, method)(a, npr, s, n, n, seed=2, keep_basis=True)
    basis = res.sketch_basis
    lc = _dense_logm(q) - res.shift_c * np.eye(n)
    g = rademacher(2, n, s, npr)
    u = g - basis @ (basis.T @ g)
    tr_s = sum(basis[:, i] @ lc @ basis[:, i] for i in range(s))
    tr_r = sum(u[:, j] @ lc @ u[:, j] for j in range(r)) / r
    assert res.tr_sketch == pytest.approx(tr_s, rel=1e-10, abs=1e-10)
    assert res.tr_resid == pytest.approx(tr_r, rel=1e-10, abs=1e-10)
    assert res.logdet == pytest.approx(n * res.shift_c + tr_s + tr_r, rel=1e-12)
    np.testing.assert_allclose(res.probe_norm2[s:], np.sum(u * u, axis=0), rtol=1e-12)


def test_osa_iop_sketch_orth_of_log_image():
    # OSA-IOP's basis spans L_c S (Alg 2), not Q S: check against the dense
    # image when Alg 1 is exact (m = n, full window).
    a = W.from_dense(W.random_spd_dense(20, seed=32, lo=0.3, hi=5.0))
    n, s = a.n, 4
    res = O.osa_iop(a, 9, s, n, n, seed=5, keep_basis=True)
    lc = _dense_logm(a.to_dense()) - res.shift_c * np.eye(n)
    y = lc @ rademacher(5, n, 0, s)
    qf, rf = np.linalg.qr(y)
    qf = qf * np.sign(np.diag(rf))[None, :]
    np.testing.assert_allclose(res.sketch_basis, qf, atol=1e-10)


@pytest.mark.parametrize("method", ["oslq", "osa_iop"])
def test_unbiased_over_seeds(method):
    # Hutch++ is unbiased given exact quadratic forms (E[g g^T] = I), so the
    # mean over seeds must approach log det Q; a wrong residual weight or a
    # dropped term shows up as a bias many standard errors wide.
    n = 10
    q = W.random_spd_dense(n, seed=12, lo=0.2, hi=6.0)
    a = W.from_dense(q)
    exact = O.dense_logdet(a)
    fn = getattr(O, method)
    est = np.array([fn(a, 5, 2, n, n, seed=sd).logdet for sd in range(300)])
    se = est.std(ddof=1) / math.sqrt(est.size)
    assert abs(est.mean() - exact) < 4.0 * se + 1e-9
    assert se > 0


def test_slq_is_sketch_rank_zero():
    a = W.lap2d(8, 0.5)
    e1 = O.slq(a, 6, 10, 2, seed=4)
    e2 = O.oslq(a, 6, 0, 10, 2, seed=4)
    assert e1.logdet == e2.logdet and e1.tr_sketch == 0.0
    assert e1.probe_norm2 == [float(a.n)] * 6  # ||g||^2 = n for Rademacher g


def test_breakdown_reports_steps():
    d = np.repeat(np.array([0.5, 1.0, 2.0]), 10)
    a = W.diag_matrix(d)
    res = O.oslq(a, 4, 1, 10, 10, seed=0)
    assert res.probe_steps == [3, 3, 3, 3]
    # with the Krylov space exhausted the quadratic forms are exact
    lc = np.diag(np.log(d) - res.shift_c)
    g = rademacher(0, a.n, 1, 4)
    basis = O.oslq(a, 4, 1, 10, 10, seed=0, keep_basis=True).sketch_basis
    u = g - basis @ (basis.T @ g)
    ref = a.n * res.shift_c + basis[:, 0] @ lc @ basis[:, 0] + sum(u[:, j] @ lc @ u[:, j] for j in range(3)) / 3
    assert res.logdet == pytest.approx(ref, rel=1e-12)


def test_laplacian_estimates_near_closed_form():
    # estimator accuracy (not parity): the 64x64 case is within the error
    # magnitudes of the paper's Table 3
    a = W.lap2d(64, 0.1)
    exact = W.lap2d_exact_logdet(64, 0.1)
    assert exact == pytest.approx(5018.30909251356, rel=1e-13)
    e = O.oslq(a, 30, 10, 30, 30, seed=0)
    assert abs(e.logdet / exact - 1) < 1e-2
    e = O.osa_iop(a, 30, 10, 30, 2, seed=0)
    assert abs(e.logdet / exact - 1) < 1e-2


def test_not_spd_detected():
    a = W.diag_matrix([-1.0, 2.0, 3.0, 4.0])
    with pytest.raises(O.NotSPDError):
        O.oslq(a, 2, 0, 4, 4, seed=0)


def test_parameter_checks():
    a = W.lap2d(4, 0.1)
    with pytest.raises(ValueError):
        O.oslq(a, 5, 5, 4, 2, seed=0)      # r = 0
    with pytest.raises(ValueError):
        O.oslq(a, 30, 17, 4, 2, seed=0)    # s > n
    with pytest.raises(ValueError):
        O.osa_iop(a, 5, 1, 0, 2, seed=0)   # m = 0


# ---------------------------------------------------------------------------
# So-SLQ (the Section 4 comparator) and Gaussian probes
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dist", [O.PROBE_RADEMACHER, O.PROBE_GAUSSIAN])
def test_so_slq_captures_a_rank_k_traced_operator(dist):
    # Q = diag(d) with four eigenvalues below 1 and the rest equal to 1:
    # lambda_hi = 1, so J = Q, c = 0 and log J has rank 4.  The dominant rank-4
    # subspace of Y = log(J) S is span(e_1..e_4); the basis runs see exact
    # Krylov spaces (5 distinct eigenvalues <= m), every residual probe is
    # projected onto the kernel of log J, and the estimate is exact.  Keeping
    # the weakest singular directions instead, or a wrong shift, fails.  The
    # basis vectors carry rounding-level components on the eigenvalue-1
    # coordinates; tol 1e-8 ends their runs at the exhausted Krylov space.
    # (The first four rows of the 12 sketch columns have full rank for seed 3.)
    d = np.concatenate([[0.01, 0.02, 0.05, 0.1], np.ones(36)])
    a = W.diag_matrix(d)
    assert np.linalg.matrix_rank(O.probes(3, 40, 0, 12, dist)[:4]) == 4
    res = O.so_slq(a, 18, 12, 4, 10, 10, 3, tol=1e-8, dist=dist, keep_basis=True)
    exact = float(np.sum(np.log(d)))
    assert res.logdet == pytest.approx(exact, rel=1e-10, abs=1e-10)
    assert abs(res.tr_resid) < 1e-10
    proj = res.sketch_basis @ res.sketch_basis.T
    np.testing.assert_allclose(proj[:4, :4], np.eye(4), atol=1e-10)
    assert np.abs(proj[4:, :]).max() < 1e-10


def test_so_slq_full_basis_is_exact():
    # k = q = n with m = n and full orthogonalisation: the basis spans R^n, the
    # residual vanishes and every quadratic form is exact
    a = W.from_dense(W.random_spd_dense(6, seed=4, lo=0.2, hi=6.0))
    res = O.so_slq(a, 7, 6, 6, 6, 6, 2, dist=O.PROBE_GAUSSIAN)
    assert res.logdet == pytest.approx(O.dense_logdet(a), rel=1e-10)
    assert abs(res.tr_resid) < 1e-10


def test_so_slq_parameter_checks():
    a = W.lap2d(8, 0.1)
    with pytest.raises(ValueError):
        O.so_slq(a, 10, 4, 5, 8, 2, 0)      # k > q
    with pytest.raises(ValueError):
        O.so_slq(a, 4, 4, 2, 8, 2, 0)       # no residual probe
    with pytest.raises(ValueError):
        O.so_slq(a, 10, 0, 0, 8, 2, 0)      # no sketch


@pytest.mark.parametrize("method", ["oslq", "osa_iop"])
def test_gaussian_probes_full_sketch_is_exact(method):
    # Hutch++ exactness does not depend on the probe distribution
    a = W.from_dense(W.random_spd_dense(8, seed=9, lo=0.3, hi=6.0))
    fn = getattr(O, method)
    res = fn(a, 9, 8, 8, 8, 1, dist=O.PROBE_GAUSSIAN)
    assert res.logdet == pytest.approx(O.dense_logdet(a), rel=1e-9)


# ---------------------------------------------------------------------------
# orth() of the sketch image (Alg 2, Alg 3: "orthonormal basis via QR"),
# including the reading for a rank-deficient image.
# ---------------------------------------------------------------------------
from oracle.estimators import RANK_RTOL, _orth  # noqa: E402


def _check_basis(q, y, kept):
    """q: the kept columns orthonormal, spanning range(y), upper-triangular
    positive-diagonal factor q^T y on the kept columns, zero elsewhere."""
    n, s = y.shape
    dropped = [j for j in range(s) if j not in kept]
    assert np.all(q[:, dropped] == 0.0)
    qk = q[:, kept]
    np.testing.assert_allclose(qk.T @ qk, np.eye(len(kept)), atol=1e-12)
    r = qk.T @ y[:, kept]
    np.testing.assert_allclose(np.tril(r, -1), 0.0, atol=1e-10)
    assert np.all(np.diag(r) > 0)
    # every column of y (kept or not) lies in span(qk)
    np.testing.assert_allclose(qk @ (qk.T @ y), y, atol=1e-9 * max(1.0, np.abs(y).max()))


def test_orth_full_rank_is_positive_diagonal_qr():
    rng = np.random.default_rng(3)
    y = rng.standard_normal((40, 7))
    _check_basis(_orth(y), y, list(range(7)))


def test_orth_drops_dependent_columns_in_order():
    rng = np.random.default_rng(4)
    a, b, c = rng.standard_normal((3, 50))
    y = np.column_stack([a, b, a + 2.0 * b, np.zeros(50), c, -3.0 * c + b])
    q = _orth(y)
    _check_basis(q, y, [0, 1, 4])


def test_orth_threshold_is_relative_to_the_column():
    rng = np.random.default_rng(5)
    a = rng.standard_normal(60)
    e = rng.standard_normal(60)
    e -= a * (a @ e) / (a @ a)
    e /= np.linalg.norm(e)
    scale = 1e5  # the test is relative to ||y_j||, not to ||Y||
    for eps, kept in ((1e-3, [0, 1]), (3.0 * RANK_RTOL, [0, 1]), (1e-9, [0])):
        col = scale * (a / np.linalg.norm(a) + eps * e)
        y = np.column_stack([a, col])
        q = _orth(y)
        assert [j for j in range(2) if np.any(q[:, j])] == kept, eps
        _check_basis(q, y, kept)


def test_osa_iop_exact_with_rank_deficient_sketch_image():
    # rank(L_c) = 3 < s = 5: Y = L_c S has rank 3, two sketch columns are
    # dropped, and Hutch++ is still exact (A spans range(L_c), every residual
    # form vanishes); the two dropped runs report K = 0, norm 0, no steps
    d = np.concatenate([np.full(27, 0.2), [0.6, 1.7, 3.1]])
    a = W.diag_matrix(d)
    s = 5
    seed = next(sd for sd in range(200)
                if np.linalg.matrix_rank(rademacher(sd, 30, 0, s)[27:, :]) == 3)
    res = O.osa_iop(a, n_probes=8, sketch_rank=s, krylov_steps=10, iop_window=2, seed=seed)
    assert res.logdet == pytest.approx(float(np.sum(np.log(d))), rel=1e-10)
    assert abs(res.tr_resid) < 1e-10
    kept = [i for i in range(s) if res.probe_norm2[i] > 0]
    assert len(kept) == 3
    for i in range(s):
        if i not in kept:
            assert res.probe_K[i] == 0.0 and res.probe_steps[i] == 0


def test_oslq_singular_sketch_matches_dense_split():
    # a singular 6 x 6 sign sketch (rank 5): the basis has 5 columns; with
    # m = n and the full window every quadratic form is exact, so the estimate
    # equals the Hutch++ split evaluated densely with an orthonormal basis of
    # range(J S) from the SVD (tr(A^T L A) and the residual depend on span(A)
    # only) and L = logm(J) - c I
    import scipy.linalg
    n = 6
    seed = next(sd for sd in range(200)
                if np.linalg.matrix_rank(rademacher(sd, n, 0, n)) == n - 1)
    a = W.from_dense(W.random_spd_dense(n, seed=11, lo=0.3, hi=4.0))
    npr = n + 3
    res = O.oslq(a, npr, n, n, n, seed)
    qd = a.to_dense()
    lo, hi = O.spectral_interval(a)
    alpha, c = O.oslq_scaling(lo, hi)
    jm = qd / alpha
    lm = np.real(scipy.linalg.logm(jm))
    y = jm @ rademacher(seed, n, 0, n)
    u, sv, _ = np.linalg.svd(y)
    basis = u[:, :int(np.sum(sv > 1e-10 * sv[0]))]
    assert basis.shape[1] == n - 1
    tr_sketch = float(np.trace(basis.T @ lm @ basis))
    g = rademacher(seed, n, n, npr)
    uu = g - basis @ (basis.T @ g)
    tr_resid = float(np.sum(uu * (lm @ uu))) / (npr - n)
    assert res.tr_sketch == pytest.approx(tr_sketch, rel=1e-9, abs=1e-10)
    assert res.tr_resid == pytest.approx(tr_resid, rel=1e-9, abs=1e-10)
    assert res.logdet == pytest.approx(n * c + tr_sketch + tr_resid, rel=1e-10)
    assert sum(1 for i in range(n) if res.probe_norm2[i] > 0) == n - 1
