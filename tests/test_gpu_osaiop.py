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
