"""GPU parity of the FP16-vector precision (LD_PREC_HALF) against the CPU FP64
oracle.

The Krylov vectors are stored in IEEE FP16 with power-of-two block scales;
products sum in FP32 (FP64 for FP64 values), inner products and norms in
FP64.  Gate: |dlogdet| / |logdet| <= 1e-4 against the oracle, as for the
FP32-vector precision, on every method, probe distribution, value type and
block shape (ragged probe counts that are not a multiple of the 8-value
chunk), and on operators whose norm forces a block scale below 1.  Start
norms come from FP64 values and must match the oracle to rounding.  The
precision is accepted only where it holds that gate (spectral bound ratio
at most 512, windows up to 4): every matrix here lies inside that range, and
the refusals outside it are tested too.
"""
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


def _rel(x, ref):
    return abs(x - ref) / abs(ref)


def _half_vs_oracle(L, ctx, a, ref, params, vt=None, lo_hint=0.0, rtol=1e-4):
    vt = L.LD_VT_FP32 if vt is None else vt
    h = ctx.matrix(a, vt=vt, lo_hint=lo_hint)
    try:
        res, det = L.ld_estimate_detail(h, params, n=a.n)
        r64 = L.ld_estimate_ex(h, L.make_params(
            params.n_probes, params.sketch_rank, params.krylov_steps, params.iop_window,
            params.seed, method=params.method, precision=L.LD_PREC_FP64, tol=params.tol,
            probe_dist=params.probe_dist, subspace_rank=params.subspace_rank,
            adapt_tol=params.adapt_tol, adapt_every=params.adapt_every))
    finally:
        ctx.release(h)
    rel = _rel(res.logdet, ref.logdet)
    print(f"  half {res.logdet!r} fp64 {r64.logdet!r} oracle {ref.logdet!r} rel {rel:.3e}",
          flush=True)
    assert np.isfinite(res.logdet)
    assert rel <= rtol
    assert _rel(res.logdet, r64.logdet) <= rtol
    return res, det


@pytest.mark.parametrize("npr,s", [(96, 32), (13, 4), (30, 10), (8, 0)])
def test_half_oslq_lap3d(L, ctx, npr, s):
    a = W.lap3d(26, 0.05)
    m, k, seed = 30, 2, 3
    _announce(f"half oslq {a.name} n={a.n} probes={npr} s={s} m={m} k={k}")
    ref = oracle.oslq(a, npr, s, m, k, seed)
    p = L.make_params(npr, s, m, k, seed, precision=L.LD_PREC_HALF)
    res, det = _half_vs_oracle(L, ctx, a, ref, p)
    np.testing.assert_allclose(det["probe_norm2"], ref.probe_norm2, rtol=1e-10)


@pytest.mark.parametrize("npr,s,k", [(40, 8, 4), (96, 32, 3)])
def test_half_oslq_any_lanes_wide_window(L, ctx, npr, s, k):
    # 5 or 12 chunks per row: the FP16 product and update on L = 5 (12 rows
    # per wave) or L = 12 lanes per row (not powers of two), with windows of
    # 3 and 4 (two inner products fused into the product)
    a = W.lap3d(26, 0.05)
    m, seed = 30, 8
    _announce(f"half oslq {a.name} n={a.n} probes={npr} s={s} m={m} k={k}")
    ref = oracle.oslq(a, npr, s, m, k, seed)
    p = L.make_params(npr, s, m, k, seed, precision=L.LD_PREC_HALF)
    _half_vs_oracle(L, ctx, a, ref, p)


@pytest.mark.parametrize("vt_name", ["FP64", "FP32", "BF16"])
def test_half_value_types(L, ctx, vt_name):
    a = W.er_laplacian(20000, 120000, seed=6, shift=0.5)
    if vt_name == "BF16":
        # the oracle runs on the matrix a bfloat16-valued product multiplies:
        # the values rounded once to bfloat16 (the library's rounding of the
        # already rounded values is exact)
        a = W.round_values_bf16(a)
    vt = getattr(L, "LD_VT_" + vt_name)
    _announce(f"half oslq {a.name} values {vt_name}")
    ref = oracle.oslq(a, 24, 8, 25, 2, 11)
    p = L.make_params(24, 8, 25, 2, 11, precision=L.LD_PREC_HALF)
    _half_vs_oracle(L, ctx, a, ref, p, vt=vt)


def test_half_wendland_with_hint(L, ctx):
    a = W.wendland(8000, 40.0, 0.1, seed=2)
    _announce(f"half oslq {a.name} with lambda_lo hint")
    ref = oracle.oslq(a, 30, 10, 30, 2, 5, lo_hint=0.1)
    p = L.make_params(30, 10, 30, 2, 5, precision=L.LD_PREC_HALF)
    _half_vs_oracle(L, ctx, a, ref, p, lo_hint=0.1)


def test_half_refuses_wide_spectral_interval(L, ctx):
    # a Wendland covariance with nugget 1e-2 (bound ratio ~1400): many
    # eigenvalues sit near the nugget and FP16 storage would move the estimate
    # by more than 1e-4, so the precision is refused; AUTO takes FP32 vectors
    # (the ratio is below 4096)
    a = W.wendland(8000, 40.0, 1e-2, seed=2)
    h = ctx.matrix(a, vt=L.LD_VT_FP32, lo_hint=1e-2)
    try:
        lo, hi = L.ld_matrix_bounds(h)
        _announce(f"half refuses {a.name} ratio {hi / lo:.0f}")
        assert 512 * lo < hi <= 4096 * lo
        p = L.make_params(30, 10, 30, 2, 5, precision=L.LD_PREC_HALF)
        with pytest.raises(L.LdError) as ei:
            L.ld_estimate_ex(h, p)
        assert ei.value.status == L.LD_E_INVALID_ARG
        with pytest.raises(L.LdError) as ei:
            L.ld_submit(h, p)
        assert ei.value.status == L.LD_E_INVALID_ARG
        auto = L.ld_estimate_ex(h, L.make_params(30, 10, 30, 2, 5, precision=L.LD_PREC_AUTO))
        mixed = L.ld_estimate_ex(h, L.make_params(30, 10, 30, 2, 5, precision=L.LD_PREC_MIXED))
        assert auto.logdet == mixed.logdet
    finally:
        ctx.release(h)


@pytest.mark.parametrize("k", [2, 4])
def test_half_osa_iop(L, ctx, k):
    a = W.lap2d(90, 0.05)
    _announce(f"half osa-iop {a.name} k={k}")
    ref = oracle.osa_iop(a, 30, 10, 20, k, 7)
    p = L.make_params(30, 10, 20, k, 7, method=L.LD_METHOD_OSA_IOP, precision=L.LD_PREC_HALF)
    _half_vs_oracle(L, ctx, a, ref, p)


def test_half_so_slq(L, ctx):
    a = W.lap3d(20, 0.05)
    _announce(f"half so-slq {a.name}")
    ref = oracle.so_slq(a, 40, 30, 10, 25, 2, 13)
    p = L.make_params(40, 30, 25, 2, 13, method=L.LD_METHOD_SO_SLQ, precision=L.LD_PREC_HALF,
                      subspace_rank=10)
    _half_vs_oracle(L, ctx, a, ref, p)


def test_half_gaussian_and_adaptive(L, ctx):
    a = W.lap3d(22, 0.05)
    _announce(f"half oslq {a.name} Gaussian probes, adaptive dimension")
    ref = oracle.oslq(a, 32, 8, 40, 2, 21, dist=oracle.PROBE_GAUSSIAN, adapt_tol=1e-6,
                      adapt_every=5)
    p = L.make_params(32, 8, 40, 2, 21, precision=L.LD_PREC_HALF,
                      probe_dist=L.LD_PROBE_GAUSSIAN, adapt_tol=1e-6, adapt_every=5)
    _half_vs_oracle(L, ctx, a, ref, p)


@pytest.mark.parametrize("factor", [1e3, 1e-3])
def test_half_operator_scale(L, ctx, factor):
    # with lambda_lo >= 1 the product runs on Q itself: a large norm forces a
    # block scale below 1; a tiny matrix takes the lambda_lo < 1 branch
    # (Q / lambda_hi) whatever its magnitude
    base = W.lap2d(70, 0.5)
    a = W.Csr(n=base.n, row_ptr=base.row_ptr, col_idx=base.col_idx,
              values=base.values * factor, name=f"{base.name}_x{factor:g}")
    _announce(f"half oslq {a.name} (operator scaled by {factor:g})")
    ref = oracle.oslq(a, 24, 8, 25, 2, 17)
    p = L.make_params(24, 8, 25, 2, 17, precision=L.LD_PREC_HALF)
    _half_vs_oracle(L, ctx, a, ref, p)


def test_half_deterministic_and_served(L, ctx):
    a = W.lap3d(24, 0.05)
    p = L.make_params(40, 12, 20, 2, 4, precision=L.LD_PREC_HALF)
    _announce(f"half determinism and serving {a.name}")
    h = ctx.matrix(a, vt=L.LD_VT_FP32)
    try:
        r1 = L.ld_estimate_ex(h, p).logdet
        r2 = L.ld_estimate_ex(h, p).logdet
        assert r1 == r2
        tickets = [L.ld_submit(h, p) for _ in range(3)]
        served = [L.ld_wait(ctx.handle, t).logdet for t in tickets]
        assert served == [r1] * 3
    finally:
        ctx.release(h)


def test_half_rejects_long_windows(L, ctx):
    # classical Gram-Schmidt over more than 4 FP16-rounded window vectors can
    # lose stability (an indefinite T on 128^3 sketch runs with window 8)
    a = W.lap2d(30, 0.1)
    h = ctx.matrix(a)
    try:
        for method in (L.LD_METHOD_OSLQ, L.LD_METHOD_OSA_IOP):
            _announce(f"half rejects window 5, method {method}")
            with pytest.raises(L.LdError) as ei:
                L.ld_estimate_ex(h, L.make_params(12, 4, 10, 5, 1, method=method,
                                                  precision=L.LD_PREC_HALF))
            assert ei.value.status == L.LD_E_INVALID_ARG
        assert np.isfinite(L.ld_estimate_ex(h, L.make_params(12, 4, 10, 4, 1,
                                                             precision=L.LD_PREC_HALF)).logdet)
    finally:
        ctx.release(h)


def test_auto_precision_choice(L, ctx):
    # LD_PREC_AUTO: FP32 vectors when lambda_hi <= 4096 lambda_lo, FP64
    # otherwise, never FP16 (whatever the window); the result is bitwise the
    # chosen precision's
    for shift, expect in ((0.5, L.LD_PREC_MIXED), (1e-2, L.LD_PREC_MIXED),
                          (1e-4, L.LD_PREC_FP64)):
        a = W.lap2d(60, shift)
        h = ctx.matrix(a, vt=L.LD_VT_FP32, lo_hint=shift)
        try:
            lo, hi = L.ld_matrix_bounds(h)
            _announce(f"auto precision {a.name} ratio {hi / lo:.1f}")
            assert (hi <= 4096 * lo) == (expect == L.LD_PREC_MIXED)
            for k in (2, 5):
                auto = L.ld_estimate_ex(h, L.make_params(20, 6, 20, k, 8,
                                                         precision=L.LD_PREC_AUTO)).logdet
                ref = L.ld_estimate_ex(h, L.make_params(20, 6, 20, k, 8,
                                                        precision=expect)).logdet
                assert auto == ref
        finally:
            ctx.release(h)
