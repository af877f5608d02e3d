"""GPU parity of the Gauss quadrature reduction and of the adaptive Krylov
dimension against the CPU FP64 oracle.

The library forms each run's K = e1^T log(T) e1 by the trapezoidal rule on
the Stieltjes integral of log when T's spectrum lies inside the operator's
spectral interval, and by Golub-Welsch otherwise; the oracle diagonalises T
(numpy eigh).  The adaptive rule stops a run at the first check t (a multiple
of adapt_every below m) where |K_t - K_{t - every}| <= adapt_tol |K_t|.  Per
run: stopping dimension exact, K within 1e-8; logdet within 1e-6 (FP64).
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


def _case(L, ctx, a, method, npr, s, m, k, seed, adapt_tol, every, lo_hint=0.0, kb=0,
          prec=None, rtol=1e-6):
    prec = L.LD_PREC_FP64 if prec is None else prec
    print(f"\n[case] {method} adaptive {a.name} n={a.n} probes={npr} s={s} m={m} k={k} "
          f"tol={adapt_tol} every={every} prec={prec}", flush=True)
    if method == "so_slq":
        ref = oracle.so_slq(a, npr, s, kb, m, k, seed, lo_hint=lo_hint, adapt_tol=adapt_tol,
                            adapt_every=every)
        mc = L.LD_METHOD_SO_SLQ
    else:
        ref = oracle.oslq(a, npr, s, m, k, seed, lo_hint=lo_hint, adapt_tol=adapt_tol,
                          adapt_every=every)
        mc = L.LD_METHOD_OSLQ
    h = ctx.matrix(a, vt=L.LD_VT_FP64 if prec == L.LD_PREC_FP64 else L.LD_VT_FP32,
                   lo_hint=lo_hint)
    try:
        p = L.make_params(npr, s, m, k, seed, method=mc, precision=prec, adapt_tol=adapt_tol,
                          adapt_every=every, subspace_rank=kb)
        res, det = L.ld_estimate_detail(h, p, n=a.n)
    finally:
        ctx.release(h)
    rel = abs(res.logdet - ref.logdet) / abs(ref.logdet)
    print(f"  gpu {res.logdet!r} oracle {ref.logdet!r} rel {rel:.3e} steps "
          f"{int(det['probe_steps'].sum())} (oracle {sum(ref.probe_steps)}) "
          f"device {res.device_ms:.2f} ms", flush=True)
    assert rel <= rtol
    if prec == L.LD_PREC_FP64:
        np.testing.assert_array_equal(det["probe_steps"], np.array(ref.probe_steps))
        np.testing.assert_allclose(det["probe_K"], ref.probe_K, rtol=1e-8, atol=1e-8)
    return ref, res, det


@pytest.mark.parametrize("adapt_tol", [0.0, 1e-4, 1e-7])
def test_oslq_adaptive_lap2d(L, ctx, adapt_tol):
    ref, res, det = _case(L, ctx, W.lap2d(45, 0.2), "oslq", 24, 8, 48, 2, 3, adapt_tol, 4)
    if adapt_tol > 0:
        assert det["probe_steps"].max() < 48


def test_oslq_adaptive_full_window_ragged(L, ctx):
    _case(L, ctx, W.lap3d(15, 0.05), "oslq", 19, 5, 40, 40, 8, 1e-6, 3)


def test_so_slq_adaptive(L, ctx):
    _case(L, ctx, W.lap2d(40, 0.1), "so_slq", 30, 12, 40, 2, 1, 1e-6, 5, kb=4)


def test_slq_adaptive_every_step(L, ctx):
    _case(L, ctx, W.er_laplacian(3000, 15000, seed=4), "oslq", 16, 0, 30, 4, 2, 1e-5, 1)


def test_adaptive_all_runs_stop_early_exit(L, ctx):
    # a loose tolerance stops every run at the second check; the remaining
    # steps are skipped (device time well below the full-depth run)
    a = W.lap3d(24, 0.5)
    ref, res, det = _case(L, ctx, a, "oslq", 20, 6, 60, 2, 4, 1e-2, 5)
    assert det["probe_steps"].max() <= 15


def test_quadrature_fallback_outside_interval(L, ctx):
    # a lower-bound hint far above the smallest eigenvalue puts Ritz values
    # below the trusted interval: those runs take the Golub-Welsch kernel
    d = np.concatenate([[1e-6, 1e-5], np.linspace(0.5, 2.0, 60)])
    a = W.diag_matrix(d)
    _case(L, ctx, a, "oslq", 10, 2, 20, 20, 1, 0.0, 5, lo_hint=0.3)


def test_adaptive_mixed(L, ctx):
    a = W.lap3d(20, 0.1)
    print("\n[case] adaptive mixed vs fp64", flush=True)
    h = ctx.matrix(a, vt=L.LD_VT_FP32)
    try:
        r64 = L.ld_estimate_ex(h, L.make_params(30, 10, 50, 2, 0, adapt_tol=1e-6, adapt_every=5))
        r32 = L.ld_estimate_ex(h, L.make_params(30, 10, 50, 2, 0, adapt_tol=1e-6, adapt_every=5,
                                                precision=L.LD_PREC_MIXED))
    finally:
        ctx.release(h)
    assert abs(r32.logdet - r64.logdet) / abs(r64.logdet) <= 1e-4


def test_adaptive_served_equals_alone(L, ctx):
    print("\n[case] adaptive served vs alone", flush=True)
    mats = [W.lap2d(60, 0.2), W.lap3d(16, 0.1)]
    ps = [L.make_params(20, 6, 40, 2, i, adapt_tol=1e-5, adapt_every=4,
                        precision=L.LD_PREC_MIXED if i % 2 else L.LD_PREC_FP64) for i in range(4)]
    with L.Context(0, max_slots=4) as c:
        hs = [c.matrix(a) for a in mats]
        alone = [L.ld_estimate_ex(hs[i % 2], p) for i, p in enumerate(ps)]
        tk = [L.ld_submit(hs[i % 2], p) for i, p in enumerate(ps)]
        got = [L.ld_wait(c.handle, t) for t in tk]
        for h in hs:
            c.release(h)
    assert [g.logdet for g in got] == [r.logdet for r in alone]
    assert [g.probe_steps for g in got] == [r.probe_steps for r in alone]
