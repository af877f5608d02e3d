"""GPU parity of the OSA-IOP path (Alg 2 with Alg 1) against the CPU oracle.

Per run: the quadratic form x^T L_c x / ||x||^2 (the GPU forms it as
sum_t g_t (log H e1)_t + log(gamma) - c, the oracle as the literal x^T y of
Alg 1's output y), the start-vector norm and the Krylov dimension; then the
log-determinant (FP64 <= 1e-6, mixed precision <= 1e-4).
"""
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


def _check(L, ctx, a, npr, s, m, k, seed, lo_hint=0.0, prec=None, vt=None, rtol=1e-6, ktol=1e-8):
    prec = L.LD_PREC_FP64 if prec is None else prec
    vt = L.LD_VT_FP64 if vt is None else vt
    print(f"\n[case] osa-iop {a.name} n={a.n} probes={npr} s={s} m={m} k={k} seed={seed} "
          f"prec={prec} vt={vt}", flush=True)
    ref = oracle.osa_iop(a, npr, s, m, k, seed, lo_hint=lo_hint)
    h = ctx.matrix(a, vt=vt, lo_hint=lo_hint)
    try:
        p = L.make_params(npr, s, m, k, seed, method=L.LD_METHOD_OSA_IOP, precision=prec)
        res, det = L.ld_estimate_detail(h, p, n=a.n, tri=True, basis=True)
    finally:
        ctx.release(h)
    rel = abs(res.logdet - ref.logdet) / abs(ref.logdet)
    print(f"  gpu {res.logdet!r} oracle {ref.logdet!r} rel {rel:.3e} device {res.device_ms:.2f} ms",
          flush=True)
    assert rel <= rtol
    assert res.scale == pytest.approx(ref.scale, rel=1e-13)
    assert res.shift_c == pytest.approx(ref.shift_c, rel=1e-13)
    if prec == L.LD_PREC_FP64:
        np.testing.assert_array_equal(det["probe_steps"], np.array(ref.probe_steps))
        np.testing.assert_allclose(det["probe_norm2"], ref.probe_norm2, rtol=1e-10)
        np.testing.assert_allclose(det["probe_K"], ref.probe_K, rtol=ktol, atol=ktol)
    return ref, res, det


@pytest.mark.parametrize("k", [2, 4])
def test_osa_iop_lap2d(L, ctx, k):
    a = W.lap2d(40, 0.1)
    _check(L, ctx, a, 24, 8, 20, k, 0)


def test_osa_iop_lap3d_full_window(L, ctx):
    a = W.lap3d(14, 1e-2)
    _check(L, ctx, a, 12, 4, 18, 18, 3)


def test_osa_iop_ragged(L, ctx):
    a = W.lap2d(29, 0.2)
    _check(L, ctx, a, 7, 3, 13, 3, 7)


def test_osa_iop_sketch_rank_zero(L, ctx):
    a = W.lap2d(25, 0.05)
    _check(L, ctx, a, 6, 0, 12, 2, 2)


def test_osa_iop_wendland_hint(L, ctx):
    a = W.wendland(2500, 30.0, 1e-2, seed=3)
    _check(L, ctx, a, 15, 5, 16, 2, 1, lo_hint=1e-2)


def test_osa_iop_breakdown(L, ctx):
    # diagonal with 4 distinct values: every run stops after at most 4 steps
    # (fewer when its start vector misses an eigenspace), the Krylov space is
    # exhausted and every quadratic form is exact
    d = np.repeat(np.array([0.3, 0.9, 2.0, 5.0]), 10)
    a = W.diag_matrix(d)
    ref, res, det = _check(L, ctx, a, 6, 2, 10, 10, 0)
    assert max(det["probe_steps"]) <= 4 and res.n_breakdowns == 6


def test_osa_iop_sketch_basis_matches(L, ctx):
    a = W.lap2d(20, 0.3)
    ref = oracle.osa_iop(a, 9, 4, 12, 2, 5, keep_basis=True)
    ref_basis = ref.sketch_basis
    h = ctx.matrix(a)
    try:
        p = L.make_params(9, 4, 12, 2, 5, method=L.LD_METHOD_OSA_IOP)
        res, det = L.ld_estimate_detail(h, p, n=a.n, basis=True)
    finally:
        ctx.release(h)
    np.testing.assert_allclose(det["sketch_basis"], ref_basis, atol=1e-10)


def test_osa_iop_mixed(L, ctx):
    a = W.lap3d(18, 1e-2)
    _check(L, ctx, a, 18, 6, 20, 2, 1, prec=L.LD_PREC_MIXED, vt=L.LD_VT_FP32, rtol=1e-4)


@pytest.mark.parametrize("nvals,m", [(5, 9), (6, 9), (5, 10), (6, 10)])
def test_osa_iop_breakdown_step_parity(L, ctx, nvals, m):
    # v1 is read on alternate steps only: runs that break down after an odd
    # or an even number of steps must still have every g_t they use (per-run
    # quadratic forms against the oracle)
    d = np.repeat(np.geomspace(0.3, 5.0, nvals), 8)
    a = W.diag_matrix(d)
    ref, res, det = _check(L, ctx, a, 9, 3, m, 2, 3)
    assert max(det["probe_steps"]) <= nvals and res.n_breakdowns >= 1


@pytest.mark.parametrize("m,k", [(7, 2), (8, 2), (7, 4), (8, 4)])
def test_osa_iop_step_count_parity(L, ctx, m, k):
    # an odd or even number of steps (the last step reads v1 or not)
    _check(L, ctx, W.lap2d(24, 0.2), 12, 4, m, k, 11)


def test_osa_iop_window_8_small(L, ctx):
    # window 8 (the largest of the 128^3 grid) at a size the oracle runs in
    # seconds, FP64 per run and mixed precision
    a = W.lap3d(18, 1e-2)
    _check(L, ctx, a, 30, 10, 24, 8, 5, ktol=1e-8)
    _check(L, ctx, a, 30, 10, 24, 8, 5, prec=L.LD_PREC_MIXED, vt=L.LD_VT_FP32, rtol=1e-4)


# ---------------------------------------------------------------------------
# Two-pass sketch image (sketch_passes = 2): the sketch-image runs go twice
# through a ring of min(k, m) + 9 blocks, the first time for H, the second
# adding each basis vector into Y before its block is reused.  The same
# kernels in the same order give the same vectors, and the batched FMA chain
# of the combination continues from the stored partial sums, so the estimate
# is bitwise the one-pass estimate over the kept basis.
# ---------------------------------------------------------------------------
def _two_pass_pair(L, ctx, a, p1, vt, lo_hint=0.0):
    import ctypes
    p2 = type(p1).from_buffer_copy(p1)
    p2.sketch_passes = 2
    h = ctx.matrix(a, vt=vt, lo_hint=lo_hint)
    try:
        r1, d1 = L.ld_estimate_detail(h, p1, n=a.n, tri=True)
        r2, d2 = L.ld_estimate_detail(h, p2, n=a.n, tri=True)
        b1, b2 = L.ld_request_bytes(h, p1), L.ld_request_bytes(h, p2)
    finally:
        ctx.release(h)
    print(f"  one pass {r1.logdet!r} ({b1} B)  two passes {r2.logdet!r} ({b2} B)", flush=True)
    assert r2.logdet == r1.logdet
    assert r2.tr_sketch == r1.tr_sketch and r2.tr_resid == r1.tr_resid
    assert r2.probe_steps == r1.probe_steps
    for key in ("probe_K", "probe_norm2", "probe_steps", "tri_alpha", "tri_beta"):
        np.testing.assert_array_equal(d2[key], d1[key])
    return r1, b1, b2


@pytest.mark.parametrize("prec_name,m,k", [("FP64", 1, 2), ("FP64", 7, 2), ("FP64", 8, 2),
                                           ("FP64", 11, 2), ("FP64", 25, 4), ("FP64", 20, 8),
                                           ("MIXED", 25, 2), ("HALF", 30, 3)])
def test_two_pass_sketch_is_bitwise_one_pass(L, ctx, prec_name, m, k):
    # m = 1: no second-pass step, v_1 alone; m = 7, 8: below and at one
    # combine batch; m = 11: the ring of window 2 (11 blocks) wraps; m = 25,
    # window 4: the ring wraps twice; window 8
    a = W.lap2d(60, 0.05)
    prec = getattr(L, "LD_PREC_" + prec_name)
    vt = L.LD_VT_FP64 if prec_name == "FP64" else L.LD_VT_FP32
    seed = 3
    print(f"\n[case] two-pass osa-iop {a.name} m={m} k={k} {prec_name}", flush=True)
    p1 = L.make_params(30, 10, m, k, seed, method=L.LD_METHOD_OSA_IOP, precision=prec)
    r1, b1, b2 = _two_pass_pair(L, ctx, a, p1, vt)
    ref = oracle.osa_iop(a, 30, 10, m, k, seed)
    tol = 1e-6 if prec_name == "FP64" else 1e-4
    assert abs(r1.logdet - ref.logdet) <= tol * abs(ref.logdet)
    # the sketch phase shrinks from m + 1 blocks of s columns to min(k, m) + 9;
    # the estimate phase's ring (n_probes columns) can still dominate, and the
    # two-pass run adds (m + 1) s multipliers
    assert b2 <= b1 + 8192


def test_two_pass_sketch_breakdown_and_so_slq(L, ctx):
    # sketch-image runs that break down after 4 steps (4 distinct
    # eigenvalues): later multipliers are zero and so are their coefficients
    a = W.diag_matrix(np.repeat(np.array([0.3, 0.9, 1.7, 4.0]), 400))
    print(f"\n[case] two-pass osa-iop breakdown {a.name}", flush=True)
    _two_pass_pair(L, ctx, a, L.make_params(24, 8, 15, 2, 4, method=L.LD_METHOD_OSA_IOP),
                   L.LD_VT_FP64)
    # So-SLQ builds its sketch of log J from the same runs
    b = W.lap3d(14, 0.05)
    print(f"\n[case] two-pass so-slq {b.name}", flush=True)
    _two_pass_pair(L, ctx, b, L.make_params(40, 20, 16, 2, 6, method=L.LD_METHOD_SO_SLQ,
                                            subspace_rank=8), L.LD_VT_FP64)


def test_two_pass_sketch_served_and_refused_for_oslq(L, ctx):
    a = W.lap2d(50, 0.1)
    h = ctx.matrix(a)
    try:
        ps = [L.make_params(20, 6, 14, 2, 9 + i, method=L.LD_METHOD_OSA_IOP,
                            sketch_passes=2 if i % 2 else 0) for i in range(4)]
        print("\n[case] two-pass osa-iop served with one-pass requests", flush=True)
        alone = [L.ld_estimate_ex(h, p).logdet for p in ps]
        tickets = [L.ld_submit(h, p) for p in ps]
        served = [L.ld_wait(ctx.handle, t).logdet for t in tickets]
        assert served == alone
        for bad in (L.make_params(20, 6, 14, 2, 1, sketch_passes=2),
                    L.make_params(20, 6, 14, 2, 1, method=L.LD_METHOD_OSA_IOP, sketch_passes=3)):
            with pytest.raises(L.LdError) as ei:
                L.ld_estimate_ex(h, bad)
            assert ei.value.status == L.LD_E_INVALID_ARG
    finally:
        ctx.release(h)
