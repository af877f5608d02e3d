"""GPU edge cases against the CPU FP64 oracle: the smallest sizes (n = 1..5,
a single residual probe, one Krylov step, window 1), the largest probe
blocks (128 FP64 / 256 mixed probes), a full sketch (s = n), and sizes that
leave ragged tails in every tiling (rows per chunk, 16-row MFMA tiles, 4-row
MFMA steps, 64-lane node batches)."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    from paper_2606_07004_amd import liblogdet
    liblogdet.lib()
    return liblogdet


@pytest.fixture(scope="module")
def ctx(L):
    c = L.Context(0)
    yield c
    c.close()


def _cmp(L, ctx, a, method, npr, s, m, k, seed, prec=None, rtol=1e-6, kb=0, exact=None):
    prec = L.LD_PREC_FP64 if prec is None else prec
    print(f"\n[case] {method} {a.name} n={a.n} probes={npr} s={s} m={m} k={k} prec={prec}",
          flush=True)
    if method == "oslq":
        ref = oracle.oslq(a, npr, s, m, k, seed)
        mc = L.LD_METHOD_OSLQ
    elif method == "osa_iop":
        ref = oracle.osa_iop(a, npr, s, m, k, seed)
        mc = L.LD_METHOD_OSA_IOP
    else:
        ref = oracle.so_slq(a, npr, s, kb, m, k, seed)
        mc = L.LD_METHOD_SO_SLQ
    h = ctx.matrix(a, vt=L.LD_VT_FP64 if prec == L.LD_PREC_FP64 else L.LD_VT_FP32)
    try:
        res = L.ld_estimate_ex(h, L.make_params(npr, s, m, k, seed, method=mc, precision=prec,
                                                subspace_rank=kb))
    finally:
        ctx.release(h)
    err = abs(res.logdet - ref.logdet) / max(abs(ref.logdet), 1e-300)
    print(f"  gpu {res.logdet!r} oracle {ref.logdet!r} rel {err:.2e}", flush=True)
    assert err <= rtol or abs(res.logdet - ref.logdet) <= 1e-12
    if exact is not None:
        assert res.logdet == pytest.approx(exact, rel=1e-9, abs=1e-9)
    return res


def _full_rank_seed(n):
    return next(sd for sd in range(100)
                if np.linalg.matrix_rank(oracle.rademacher(sd, n, 0, n)) == n)


@pytest.mark.parametrize("method", ["oslq", "osa_iop"])
@pytest.mark.parametrize("n", [1, 2, 5, 8])
def test_tiny_matrices(L, ctx, method, n):
    # n <= 8 with a full sketch (a seed whose n x n sign matrix is
    # nonsingular), m = n, full window: exact log-determinants
    a = W.from_dense(W.random_spd_dense(n, seed=n, lo=0.2, hi=3.0))
    exact = oracle.dense_logdet(a)
    _cmp(L, ctx, a, method, n + 1, n, n, n, _full_rank_seed(n), exact=exact)


@pytest.mark.parametrize("method", ["oslq", "osa_iop"])
def test_singular_sketch_keeps_independent_columns(L, ctx, method):
    # a singular 6 x 6 sign sketch (rank 5): orth() keeps the 5 independent
    # columns in order and leaves a zero column whose run is skipped (the
    # oracle's reading of a rank-deficient sketch image); per-run values and
    # the estimate against the oracle
    n = 6
    seed = next(sd for sd in range(200)
                if np.linalg.matrix_rank(oracle.rademacher(sd, n, 0, n)) == n - 1)
    a = W.from_dense(W.random_spd_dense(n, seed=11, lo=0.3, hi=4.0))
    npr = n + 3
    fn = oracle.oslq if method == "oslq" else oracle.osa_iop
    ref = fn(a, npr, n, n, n, seed)
    print(f"\n[case] singular sketch {method} n={n} seed={seed}", flush=True)
    h = ctx.matrix(a)
    try:
        mc = L.LD_METHOD_OSLQ if method == "oslq" else L.LD_METHOD_OSA_IOP
        res, det = L.ld_estimate_detail(h, L.make_params(npr, n, n, n, seed, method=mc), n=n)
    finally:
        ctx.release(h)
    print(f"  gpu {res.logdet!r} oracle {ref.logdet!r} rank {res.basis_rank}", flush=True)
    assert res.basis_rank == n - 1
    assert abs(res.logdet - ref.logdet) <= 1e-6 * abs(ref.logdet)
    np.testing.assert_array_equal(det["probe_steps"], np.array(ref.probe_steps))
    np.testing.assert_allclose(det["probe_norm2"], ref.probe_norm2, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(det["probe_K"], ref.probe_K, rtol=1e-8, atol=1e-10)


@pytest.mark.parametrize("prec_name", ["FP64", "MIXED"])
def test_rank_deficient_sketch_image_is_exact(L, ctx, prec_name):
    # OSA-IOP with rank(L_c) = 3 < s = 5: the sketch image Y = L_c S has rank
    # 3, two columns are dropped and Hutch++ stays exact (Alg 2 on a traced
    # operator of rank below the sketch size)
    d = np.concatenate([np.full(2997, 0.2), [0.6, 1.7, 3.1]])
    a = W.diag_matrix(d)
    s = 5
    seed = next(sd for sd in range(400)
                if np.linalg.matrix_rank(oracle.rademacher(sd, a.n, 0, s)[-3:, :]) == 3)
    ref = oracle.osa_iop(a, 8, s, 10, 2, seed)
    exact = float(np.sum(np.log(d)))
    prec = getattr(L, "LD_PREC_" + prec_name)
    print(f"\n[case] rank-deficient sketch image osa-iop n={a.n} s={s} {prec_name}", flush=True)
    h = ctx.matrix(a, vt=L.LD_VT_FP64 if prec_name == "FP64" else L.LD_VT_FP32)
    try:
        res = L.ld_estimate_ex(h, L.make_params(8, s, 10, 2, seed, method=L.LD_METHOD_OSA_IOP,
                                                precision=prec))
    finally:
        ctx.release(h)
    print(f"  gpu {res.logdet!r} oracle {ref.logdet!r} exact {exact!r} rank {res.basis_rank}",
          flush=True)
    # FP64: the dependent columns are dependent to rounding and dropped.  FP32
    # Krylov vectors leave ~1e-7 noise on each of the 2997 null-space rows of
    # Y, which can keep a dependent column as a noise direction; that
    # direction lies in the null space of L_c and adds nothing to the trace
    assert res.basis_rank == 3 if prec_name == "FP64" else 3 <= res.basis_rank <= 5
    tol = 1e-9 if prec_name == "FP64" else 1e-5
    assert res.logdet == pytest.approx(exact, rel=tol)
    assert res.logdet == pytest.approx(ref.logdet, rel=tol)


def test_multiple_of_identity_is_exact(L, ctx):
    # zero-width spectral interval: Q = q I, the estimate is n log q exactly
    a = W.diag_matrix(np.full(300, 2.5))
    for method in (L.LD_METHOD_OSLQ, L.LD_METHOD_OSA_IOP, L.LD_METHOD_SO_SLQ):
        h = ctx.matrix(a)
        try:
            r = L.ld_estimate_ex(h, L.make_params(20, 8, 10, 2, 0, method=method))
        finally:
            ctx.release(h)
        assert r.logdet == pytest.approx(300 * np.log(2.5), rel=1e-15)


def test_single_step_single_probe(L, ctx):
    a = W.lap2d(17, 0.2)
    _cmp(L, ctx, a, "oslq", 1, 0, 1, 1, 0)
    _cmp(L, ctx, a, "oslq", 3, 2, 1, 1, 4)


def test_window_one(L, ctx):
    # window 1: each new vector is orthogonalised against the newest one only.
    # OSA-IOP takes log(H) e1 of the resulting Hessenberg matrix; OSLQ's
    # tridiagonal T of such a run need not be positive definite, and both the
    # oracle and the library then report a non-positive Ritz value
    a = W.lap2d(23, 0.3)
    _cmp(L, ctx, a, "osa_iop", 9, 3, 10, 1, 2)
    with pytest.raises(oracle.NotSPDError):
        oracle.oslq(a, 9, 3, 10, 1, 2)
    h = ctx.matrix(a)
    try:
        with pytest.raises(L.LdError) as e:
            L.ld_estimate_ex(h, L.make_params(9, 3, 10, 1, 2))
        assert e.value.status == L.LD_E_NOT_SPD
    finally:
        ctx.release(h)


@pytest.mark.parametrize("prec,npr", [("fp64", 128), ("mixed", 256)])
def test_largest_probe_blocks(L, ctx, prec, npr):
    a = W.lap3d(11, 0.1)
    p = L.LD_PREC_FP64 if prec == "fp64" else L.LD_PREC_MIXED
    _cmp(L, ctx, a, "oslq", npr, npr // 4, 8, 2, 9, prec=p, rtol=1e-6 if prec == "fp64" else 1e-4)


def test_probe_limits_rejected(L, ctx):
    a = W.lap2d(20, 0.1)
    h = ctx.matrix(a)
    try:
        for p in (L.make_params(129, 10, 8, 2, 0),
                  L.make_params(257, 10, 8, 2, 0, precision=L.LD_PREC_MIXED)):
            with pytest.raises(L.LdError) as e:
                L.ld_estimate_ex(h, p)
            assert e.value.status == L.LD_E_INVALID_ARG
    finally:
        ctx.release(h)


@pytest.mark.parametrize("n", [255, 257, 1023, 4099])
def test_ragged_tails(L, ctx, n):
    # diagonal-plus-chain matrices of awkward sizes: partial chunks, partial
    # 16-row and 4-row MFMA tiles, a sketch of 13 columns
    rng = np.random.default_rng(n)
    d = rng.uniform(1.5, 3.0, n)
    dense_off = rng.uniform(-0.5, 0.5, n - 1)
    import scipy.sparse as sp
    q = sp.diags([dense_off, d, dense_off], [-1, 0, 1], format="csr")
    a = W.Csr(n=n, row_ptr=q.indptr.astype(np.int32), col_idx=q.indices.astype(np.int32),
              values=q.data.astype(np.float64), name=f"chain_{n}")
    _cmp(L, ctx, a, "oslq", 40, 13, 12, 2, 1)
    _cmp(L, ctx, a, "so_slq", 40, 13, 12, 2, 1, kb=5)


def test_m_equals_n_full_window_exact(L, ctx):
    # Krylov dimension n with full orthogonalisation on a 24 x 24 system:
    # every quadratic form exact, so with s = n the estimate is log det Q
    a = W.from_dense(W.random_spd_dense(24, seed=7, lo=0.3, hi=4.0))
    _cmp(L, ctx, a, "oslq", 25, 24, 24, 24, 0, exact=oracle.dense_logdet(a))
