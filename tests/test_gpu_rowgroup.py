"""GPU tests of the row-group product (FP32 values on FP32 Krylov vectors,
FP64 values on FP64 or FP32 ones).

A matrix created with FP32 or FP64 values whose groups of 4 consecutive rows
share most of their columns keeps, per group, the union of the rows' columns with
one value per row (zero where a row has no entry); the product can read the
groups instead of the CSR rows and gather each union column's probe row once
for the group.  A row's sum sees its nonzero terms in CSR order, so the
product's output is the CSR product's; the inner products fused into it sum
the rows in another order (FP64).  Every case pins the CSR product and then
the row-group product in the same geometry and compares the two estimates
(tightly) and each with the CPU FP64 oracle (the mixed-precision 1e-4).
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


# 6002 points: the last group holds 2 rows
NUG = 1e-2


@pytest.fixture(scope="module")
def cov():
    return W.wendland(6002, 48.0, NUG, seed=21)


def _pair(L, ctx, a, method, npr, s, m, k, seed, geoms, fp64=False, vt=None):
    fn = oracle.oslq if method == L.LD_METHOD_OSLQ else oracle.osa_iop
    ref = fn(a, npr, s, m, k, seed, lo_hint=NUG)
    h = ctx.matrix(a, vt=L.LD_VT_FP32 if vt is None else vt, lo_hint=NUG)
    # FP64 estimates: the oracle's 1e-6, and the two products' W agree to the
    # last bit (only the order of the fused FP64 inner products differs)
    tol, ptol = (1e-6, 1e-10) if fp64 else (1e-4, 1e-7)
    try:
        p = L.make_params(npr, s, m, k, seed, method=method,
                          precision=L.LD_PREC_FP64 if fp64 else L.LD_PREC_MIXED)
        # 16-byte chunks of a row
        ncolv = (npr + 3) // 4 * (2 if fp64 else 1)
        for lanes, ch, il, sched in geoms:
            got = {}
            for rg in (0, 1):
                _announce(f"row groups {rg}: method {method} fp64 {fp64} n={a.n} probes {npr} "
                          f"window {k} L={lanes} C={ch} interleave {il} schedule {sched}")
                L.ld_tune_set(h, p, lanes, ch, ncolv, 1, 1, il, 0, sched, rg)
                res = L.ld_estimate_ex(h, p)
                rel = abs(res.logdet - ref.logdet) / abs(ref.logdet)
                print(f"  logdet {res.logdet!r} rel {rel:.3e}", flush=True)
                assert rel <= tol, (rg, rel)
                assert L.ld_estimate_ex(h, p).logdet == res.logdet  # reproducible
                got[rg] = res
            a0, a1 = got[0], got[1]
            assert abs(a1.logdet - a0.logdet) <= ptol * abs(a0.logdet)
            assert abs(a1.tr_resid - a0.tr_resid) <= ptol * abs(a0.tr_resid) + 1e-9
            assert a1.probe_steps == a0.probe_steps
    finally:
        ctx.release(h)


def test_rowgroup_oslq_window2(L, ctx, cov):
    # 30 probes (8 chunks): one and two chunks per lane, both chunk mappings,
    # both step schedules
    _pair(L, ctx, cov, L.LD_METHOD_OSLQ, 30, 10, 16, 2, 3,
          [(8, 1, 0, 1), (8, 1, 1, 0), (4, 2, 0, 1), (4, 2, 1, 1), (16, 1, 0, 1)])


def test_rowgroup_oslq_wide_windows(L, ctx, cov):
    # 64 probes (16 chunks); window 4 (separate window dots) and window 10
    # (beyond one update launch: the product then fuses two inner products)
    _pair(L, ctx, cov, L.LD_METHOD_OSLQ, 64, 20, 14, 4, 5, [(16, 1, 0, 1), (8, 2, 1, 1)])
    _pair(L, ctx, cov, L.LD_METHOD_OSLQ, 30, 10, 14, 10, 6, [(8, 1, 0, 1)])


def test_rowgroup_osa_iop(L, ctx, cov):
    _pair(L, ctx, cov, L.LD_METHOD_OSA_IOP, 30, 10, 12, 2, 7, [(8, 1, 0, 1)])


def test_rowgroup_lanes_not_power_of_two(L, ctx, cov):
    # 22 probes (6 chunks): 6 lanes per group (10 groups per wave, 4 lanes
    # idle) and 3 lanes of two chunks
    _pair(L, ctx, cov, L.LD_METHOD_OSLQ, 22, 6, 12, 2, 9, [(6, 1, 0, 1), (3, 2, 1, 1)])


def test_rowgroup_fp64(L, ctx, cov):
    # FP64 values on FP64 Krylov vectors: 30 probes (16 chunks of two FP64
    # values), one and two chunks per lane, both schedules; OSA-IOP
    _pair(L, ctx, cov, L.LD_METHOD_OSLQ, 30, 10, 14, 2, 11,
          [(16, 1, 0, 1), (8, 2, 1, 1), (16, 1, 1, 0)], fp64=True)
    _pair(L, ctx, cov, L.LD_METHOD_OSA_IOP, 30, 10, 10, 2, 12, [(16, 1, 0, 1)], fp64=True)


def test_rowgroup_fp64_storage_mixed(L, ctx, cov):
    # FP64 storage: mixed runs read the FP64 values (FP64 sums) on FP32 vectors
    _pair(L, ctx, cov, L.LD_METHOD_OSLQ, 30, 10, 14, 2, 13, [(8, 1, 0, 1), (4, 2, 1, 1)],
          vt=L.LD_VT_FP64)


def _groups_by_definition(a):
    """Row groups written out from their definition: per group of 4 rows the
    sorted union of the rows' columns and, per union column, each row's value
    (0 where the row has no entry there)."""
    rp, ci, va = a.row_ptr, a.col_idx, a.values
    gp, cols, vals = [0], [], []
    for g in range((a.n + 3) // 4):
        rows = range(4 * g, min(a.n, 4 * g + 4))
        u = np.unique(np.concatenate([ci[rp[r]:rp[r + 1]] for r in rows]))
        v = np.zeros((len(u), 4))
        for j, r in enumerate(rows):
            v[np.searchsorted(u, ci[rp[r]:rp[r + 1]]), j] = va[rp[r]:rp[r + 1]]
        gp.append(gp[-1] + len(u))
        cols.append(u)
        vals.append(v)
    return np.array(gp), np.concatenate(cols), np.concatenate(vals)


def test_rowgroup_build_exact(L, ctx, cov):
    # the device-built groups against their definition, element by element
    gp, col, val = _groups_by_definition(cov)
    assert cov.nnz >= 2 * len(col)  # kept: at least 2 entries per union column
    for vt in (L.LD_VT_FP32, L.LD_VT_FP64):
        _announce(f"row groups built on the device, storage {vt}, n={cov.n}")
        h = ctx.matrix(cov, vt=vt, lo_hint=NUG)
        try:
            got = L.ld_debug_row_groups(h, cov.n)
            assert got is not None
            assert np.array_equal(got[0], gp)
            assert np.array_equal(got[1], col)
            assert np.array_equal(got[2], val)
        finally:
            ctx.release(h)
    _announce("no row groups on a Laplacian (1.3 entries per union column) or BF16 values")
    for a, vt in ((W.lap3d(20, 1e-2), L.LD_VT_FP32), (cov, L.LD_VT_BF16)):
        h = ctx.matrix(a, vt=vt, lo_hint=NUG if a is cov else 0.0)
        try:
            assert L.ld_debug_row_groups(h, a.n) is None
        finally:
            ctx.release(h)


def test_rowgroup_default_and_tuner(L, ctx, cov):
    npr, s, m, k, seed = 30, 10, 12, 2, 8
    h = ctx.matrix(cov, vt=L.LD_VT_FP32, lo_hint=NUG)
    try:
        p = L.make_params(npr, s, m, k, seed, precision=L.LD_PREC_MIXED)
        _announce("untuned FP32 covariance: the row-group product by default")
        base = L.ld_estimate_ex(h, p).logdet
        L.ld_tune_set(h, p, 8, 1, 8, 1, 1, 0, 0, 1, 1)
        assert L.ld_estimate_ex(h, p).logdet == base
        _announce("autotuner with row-group candidates")
        tr = L.ld_autotune(h, p, 3)
        assert tr.spmm_row_groups in (0, 1)
        assert tr.spmm_ms <= tr.spmm_default_ms
        res = L.ld_estimate_ex(h, p).logdet
        assert abs(res - base) <= 1e-7 * abs(base)
        L.ld_autotune(h, p, 0)
        assert L.ld_estimate_ex(h, p).logdet == base
        _announce("row groups refused with three chunks per lane")
        with pytest.raises(L.LdError):
            L.ld_tune_set(h, p, 4, 3, 8, 1, 1, 0, 0, 1, 1)
    finally:
        ctx.release(h)
    _announce("row groups refused where the matrix keeps none")
    for a, vt in ((W.lap3d(20, 1e-2), L.LD_VT_FP32), (cov, L.LD_VT_BF16)):
        h = ctx.matrix(a, vt=vt, lo_hint=NUG if a is cov else 0.0)
        try:
            p = L.make_params(npr, s, m, k, seed, precision=L.LD_PREC_MIXED)
            L.ld_tune_set(h, p, 8, 1, 8, 1, 1, 0, 0, 1, 0)
            with pytest.raises(L.LdError):
                L.ld_tune_set(h, p, 8, 1, 8, 1, 1, 0, 0, 1, 1)
        finally:
            ctx.release(h)
