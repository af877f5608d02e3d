"""GPU parity of the OSLQ path (Alg 3) against the CPU FP64 oracle.

Every case runs the HIP library through its C ABI and compares, element by
element, the per-run quadrature values, start-vector norms, Krylov
dimensions and tridiagonal coefficients with the oracle on the same seeded
inputs, then the assembled log-determinant.  Tolerances: FP64 mode
|dlogdet|/|logdet| <= 1e-6 (per-run values much tighter); mixed precision
(FP32 vectors and values, FP64 reductions) <= 1e-4.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

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


def _announce(msg):
    print(f"\n[case] {msg}", flush=True)


def _check_oslq(L, ctx, a, npr, s, m, k, seed, lo_hint=0.0, hi_hint=0.0,
                prec=None, vt=None, rtol=1e-6):
    prec = L.LD_PREC_FP64 if prec is None else prec
    vt = L.LD_VT_FP64 if vt is None else vt
    _announce(f"oslq {a.name} n={a.n} nnz={a.nnz} probes={npr} s={s} m={m} k={k} "
              f"seed={seed} prec={prec} vt={vt}")
    ref = oracle.oslq(a, npr, s, m, k, seed, lo_hint=lo_hint, hi_hint=hi_hint)
    h = ctx.matrix(a, vt=vt, lo_hint=lo_hint, hi_hint=hi_hint)
    try:
        p = L.make_params(npr, s, m, k, seed, method=L.LD_METHOD_OSLQ, precision=prec)
        res, det = L.ld_estimate_detail(h, p, n=a.n, tri=True)
    finally:
        ctx.release(h)
    rel = abs(res.logdet - ref.logdet) / abs(ref.logdet)
    print(f"  gpu {res.logdet!r} oracle {ref.logdet!r} rel {rel:.3e} device {res.device_ms:.3f} ms",
          flush=True)
    assert res.shift_c == pytest.approx(ref.shift_c, rel=1e-14)
    assert res.lambda_lo == pytest.approx(ref.lambda_lo, rel=1e-12)
    assert res.lambda_hi == pytest.approx(ref.lambda_hi, rel=1e-12)
    assert rel <= rtol
    return ref, res, det


def _elementwise(ref, det, s, ktol, ntol=1e-10):
    np.testing.assert_array_equal(det["probe_steps"], np.array(ref.probe_steps))
    np.testing.assert_allclose(det["probe_norm2"], ref.probe_norm2, rtol=ntol)
    np.testing.assert_allclose(det["probe_K"], ref.probe_K, rtol=ktol, atol=ktol)
    for p, (al, be) in enumerate(zip(ref.probe_alpha, ref.probe_beta)):
        me = ref.probe_steps[p]
        np.testing.assert_allclose(det["tri_alpha"][p, :me], al, rtol=ktol, atol=ktol)
        np.testing.assert_allclose(det["tri_beta"][p, :me - 1], be[:me - 1], rtol=ktol, atol=ktol)


def test_rademacher_bit_exact(L, ctx):
    _announce("rademacher n=1000 cols 3..41 seed 77")
    got = L.ld_debug_rademacher(ctx.handle, 77, 1000, 3, 41)
    ref = oracle.rademacher(77, 1000, 3, 41)
    np.testing.assert_array_equal(got, ref)
    _announce("rademacher n=70000 cols 0..5 seed 2**63+5")
    seed = 2**63 + 5
    np.testing.assert_array_equal(L.ld_debug_rademacher(ctx.handle, seed, 70000, 0, 5),
                                  oracle.rademacher(seed, 70000, 0, 5))


def test_oslq_c1_fp64_full_reorth(L, ctx):
    # 64x64 2D Laplacian + 0.1 I, 30 probes (10 + 20), 30 steps, full window
    a = W.lap2d(64, 0.1)
    ref, res, det = _check_oslq(L, ctx, a, 30, 10, 30, 30, 0)
    _elementwise(ref, det, 10, 1e-9)
    exact = W.lap2d_exact_logdet(64, 0.1)
    print(f"  estimator error vs closed form {abs(res.logdet / exact - 1):.3e}")


@pytest.mark.parametrize("k", [2, 4, 8])
def test_oslq_lap3d_windows(L, ctx, k):
    a = W.lap3d(20, 1e-2)
    ref, res, det = _check_oslq(L, ctx, a, 24, 8, 25, k, 3)
    _elementwise(ref, det, 8, 1e-8)


@pytest.mark.parametrize("prec_name,npr,k", [("FP64", 24, 10), ("MIXED", 96, 8),
                                              ("FP64", 128, 8), ("MIXED", 256, 7)])
def test_oslq_wide_window_dots(L, ctx, prec_name, npr, k):
    # windows with more than four vectors older than the two newest: their
    # inner products in one launch of up to eight, one 16-byte chunk per lane
    # (up to 64 lanes per row: 128 FP64 or 256 FP32 probes)
    a = W.lap2d(36, 0.05)
    prec = getattr(L, "LD_PREC_" + prec_name)
    vt = L.LD_VT_FP64 if prec_name == "FP64" else L.LD_VT_FP32
    tol = 1e-6 if prec_name == "FP64" else 1e-4
    ref, res, det = _check_oslq(L, ctx, a, npr, 8, 18, k, 4, prec=prec, vt=vt, rtol=tol)
    if prec_name == "FP64":
        _elementwise(ref, det, 8, 1e-8)


def test_oslq_ragged_sizes(L, ctx):
    # n not a multiple of any tile, 7 probes (padded block of 8), odd window
    a = W.lap2d(37, 0.3)
    ref, res, det = _check_oslq(L, ctx, a, 7, 2, 11, 3, 11)
    _elementwise(ref, det, 2, 1e-9)


def test_oslq_sketch_rank_zero_is_slq(L, ctx):
    a = W.lap2d(30, 0.05)
    ref, res, det = _check_oslq(L, ctx, a, 9, 0, 15, 2, 5)
    _elementwise(ref, det, 0, 1e-9)
    assert res.tr_sketch == 0.0


def test_oslq_er_graph(L, ctx):
    a = W.er_laplacian(6000, 48000, seed=0, shift=0.05)
    ref, res, det = _check_oslq(L, ctx, a, 20, 6, 20, 4, 0)
    _elementwise(ref, det, 6, 1e-8)


def test_oslq_wendland_with_hint(L, ctx):
    a = W.wendland(3000, 30.0, 1e-2, seed=2)
    ref, res, det = _check_oslq(L, ctx, a, 16, 5, 20, 2, 1, lo_hint=1e-2)
    _elementwise(ref, det, 5, 1e-8)


def test_oslq_breakdown_diag(L, ctx):
    d = np.repeat(np.array([0.5, 1.0, 2.0, 4.0]), 9)
    a = W.diag_matrix(d)
    ref, res, det = _check_oslq(L, ctx, a, 5, 1, 10, 10, 0)
    assert list(det["probe_steps"]) == [4] * 5
    assert res.n_breakdowns == 5
    assert res.logdet == pytest.approx(float(np.sum(np.log(d))), rel=0.05)


def test_oslq_deterministic(L, ctx):
    a = W.lap3d(16, 1e-1)
    h = ctx.matrix(a)
    try:
        p = L.make_params(20, 6, 15, 2, 9)
        r1 = L.ld_estimate_ex(h, p).logdet
        r2 = L.ld_estimate_ex(h, p).logdet
    finally:
        ctx.release(h)
    assert r1 == r2  # bitwise: fixed-order reductions, no atomics


@pytest.mark.parametrize("vt_name", ["LD_VT_FP32", "LD_VT_BF16"])
def test_oslq_mixed_precision(L, ctx, vt_name):
    a = W.lap3d(20, 1e-2)
    vt = getattr(L, vt_name)
    if vt == L.LD_VT_BF16:
        # BF16 storage multiplies by the matrix with its values rounded to
        # bfloat16: the oracle runs on exactly that matrix (rounded once,
        # nearest-even, on the host), so the gate measures the arithmetic of
        # the BF16-valued product and FP32 vectors, not the change of matrix
        a = W.round_values_bf16(W.er_laplacian(6000, 48000, seed=3, shift=0.05))
    _check_oslq(L, ctx, a, 24, 8, 25, 2, 3, prec=L.LD_PREC_MIXED, vt=vt, rtol=1e-4)


def test_bf16_storage_rounds_nearest_even(L, ctx):
    # the library rounds FP64 values to bfloat16 once, nearest-even: a matrix
    # given unrounded and the same matrix rounded on the host beforehand give
    # bitwise the same estimate in BF16 storage (both with the same spectral
    # interval: the Gershgorin bounds come from the FP64 values, which differ)
    a = W.er_laplacian(6000, 48000, seed=3, shift=0.05)
    rows = np.repeat(np.arange(a.n), np.diff(a.row_ptr))
    jit = 1.0 + 1e-3 * np.sin(rows + a.col_idx.astype(np.int64))  # symmetric in (row, col)
    a = W.Csr(n=a.n, row_ptr=a.row_ptr, col_idx=a.col_idx, values=a.values * jit,
              name=a.name + "_jit")
    ar = W.round_values_bf16(a)
    assert not np.array_equal(a.values, ar.values)
    _announce(f"bf16 rounding {a.name}")
    p = L.make_params(16, 5, 15, 2, 7, precision=L.LD_PREC_MIXED)
    out = []
    for m in (a, ar):
        h = ctx.matrix(m, vt=L.LD_VT_BF16, lo_hint=0.05, hi_hint=64.0)
        try:
            out.append(L.ld_estimate_ex(h, p).logdet)
        finally:
            ctx.release(h)
    assert out[0] == out[1]


def test_error_paths(L, ctx):
    _announce("error paths")
    a = W.lap2d(8, 0.1)
    h = ctx.matrix(a)
    try:
        with pytest.raises(L.LdError) as e:
            L.ld_estimate_ex(h, L.make_params(5, 5, 4, 2, 0))       # r = 0
        assert e.value.status == L.LD_E_INVALID_ARG
        with pytest.raises(L.LdError) as e:
            L.ld_estimate_ex(h, L.make_params(10, 2, 65, 2, 0))     # m > n
        assert e.value.status == L.LD_E_INVALID_ARG
        with pytest.raises(L.LdError) as e:
            L.ld_estimate_ex(h, L.make_params(10, 2, 4, 0, 0))      # k = 0
        assert e.value.status == L.LD_E_INVALID_ARG
    finally:
        ctx.release(h)
    bad = W.diag_matrix([1.0, -2.0, 3.0])
    with pytest.raises(L.LdError) as e:
        ctx.matrix(bad)
    assert e.value.status == L.LD_E_NOT_SPD
    with pytest.raises(L.LdError) as e:
        L.ld_create_csr(ctx.handle, 3, 3, [0, 1, 2, 3], [0, 2, 1], [1.0, 1.0, 1.0])
    assert e.value.status in (L.LD_E_BAD_CSR, L.LD_E_NOT_SPD)
    with pytest.raises(L.LdError) as e:
        L.ld_create_csr(ctx.handle, 2, 3, [0, 2, 3], [1, 0, 1], [1.0, 1.0, 1.0])
    assert e.value.status == L.LD_E_BAD_CSR


@pytest.mark.parametrize("s", [1, 63, 64, 65, 80])
def test_oslq_sketch_widths(L, ctx, s):
    # sketch widths around the matrix-core limit of the sketch kernels (64
    # columns): both the MFMA and the scalar Gram / triangular / projection paths
    a = W.lap2d(45, 0.3)
    ref, res, det = _check_oslq(L, ctx, a, s + 20, s, 12, 2, 5)
    _elementwise(ref, det, s, 1e-8)


@pytest.mark.parametrize("prec_name,vt_name,npr,s", [("FP64", "FP64", 110, 20),
                                                     ("MIXED", "FP32", 110, 20),
                                                     ("HALF", "FP32", 150, 21)])
def test_oslq_wide_residual_block(L, ctx, prec_name, vt_name, npr, s):
    # residual blocks wider than 64 columns and ragged against the 16-column
    # tiles: two or three sign words per row for the Rademacher residual
    # probes, several tile groups in the projection, output tiles staged in
    # LDS or stored directly depending on their size
    a = W.lap2d(50, 0.2)
    prec = getattr(L, "LD_PREC_" + prec_name)
    vt = getattr(L, "LD_VT_" + vt_name)
    ref, res, det = _check_oslq(L, ctx, a, npr, s, 14, 2, 9, prec=prec, vt=vt,
                                rtol=1e-6 if prec_name == "FP64" else 1e-4)
    # squared residual norms from the FP64 projection, before any narrowing;
    # with FP32 values the sketch product itself sees the rounded matrix
    # (2^-24 per value), which moves the sketch basis and so the norms
    np.testing.assert_allclose(det["probe_norm2"], ref.probe_norm2,
                               rtol=1e-10 if vt_name == "FP64" else 1e-6)


def test_oslq_wide_residual_block_gaussian(L, ctx):
    # Gaussian residual probes take the dense-column path of the same kernels
    a = W.lap2d(50, 0.2)
    npr, s, m, k, seed = 110, 20, 14, 2, 12
    _announce(f"oslq {a.name} Gaussian probes={npr} s={s}")
    ref = oracle.oslq(a, npr, s, m, k, seed, dist=oracle.PROBE_GAUSSIAN)
    h = ctx.matrix(a)
    try:
        p = L.make_params(npr, s, m, k, seed, probe_dist=L.LD_PROBE_GAUSSIAN)
        res, det = L.ld_estimate_detail(h, p, n=a.n)
    finally:
        ctx.release(h)
    rel = abs(res.logdet - ref.logdet) / abs(ref.logdet)
    print(f"  gpu {res.logdet!r} oracle {ref.logdet!r} rel {rel:.3e}", flush=True)
    assert rel <= 1e-6
    np.testing.assert_allclose(det["probe_norm2"], ref.probe_norm2, rtol=1e-9)
