"""GPU tests of the Krylov-step geometry autotuner (ld_autotune, ld_tune_set).

The product and update kernels sweep a probe block with L lanes per row and
C 16-byte chunks per lane.  Any usable (L, C) must give the same estimate up
to the summation order of the FP64 partial sums: every geometry is forced in
turn and compared with the CPU FP64 oracle (1e-6 FP64, 1e-4 mixed) and with
the default geometry (much tighter).  A tuned matrix must keep results
bitwise reproducible, served requests equal to the same request alone, and
a reset must restore the untuned results bit for bit.
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


def _usable(ncolv):
    return [(lanes, ch) for lanes in (1, 2, 4, 8, 16, 32, 64) for ch in (1, 2, 3, 4)
            if lanes * ch >= ncolv]


def _np2_lanes(ncolv):
    """Geometries with L lanes per row not a power of two (a wave holds
    floor(64 / L) rows, the rest of its lanes idle): the tight
    L = ceil(ncolv / C) and one with a spare lane per row."""
    out = []
    for ch in (1, 2, 3, 4):
        for lanes in (-(-ncolv // ch), -(-ncolv // ch) + 1):
            if lanes <= 64 and lanes & (lanes - 1) and (lanes, ch) not in out:
                out.append((lanes, ch))
    return out


def _splits(lanes, chunks=1):
    """Entry splits of the product that fit `lanes` column lanes in 64 (one or
    two chunks per lane)."""
    return [e for e in (1, 2, 4, 8) if lanes * e <= 64 and (e == 1 or chunks <= 2)]


def _sweep(L, ctx, a, npr, prec, vt, rtol_oracle, rtol_default, vec, k):
    s, m, seed = 6, 14, 31
    ref = oracle.oslq(a, npr, s, m, k, seed)
    h = ctx.matrix(a, vt=vt)
    try:
        p = L.make_params(npr, s, m, k, seed, method=L.LD_METHOD_OSLQ, precision=prec)
        base = L.ld_estimate_ex(h, p).logdet
        assert abs(base - ref.logdet) <= rtol_oracle * abs(ref.logdet)
        ncolv = ((npr + 3) // 4 * 4) // vec
        geoms = _usable(ncolv) + _np2_lanes(ncolv)
        cases = [(lanes, ch, e) for lanes, ch in geoms
                 for e in (_splits(lanes, ch) if lanes & (lanes - 1) == 0 else [1])]
        for i, (lanes, ch, e) in enumerate(cases):
            # the update takes the geometries in the other order, so product
            # and update differ in most cases
            ul, uc = geoms[(len(geoms) - 1 - i) % len(geoms)]
            # every other case interleaves the product's chunks over the XCDs
            il = i % 2
            _announce(f"forced geometry n={a.n} probes={npr} prec={prec} "
                      f"product L={lanes * e} C={ch} split={e} interleave={il} "
                      f"update L={ul} C={uc}")
            L.ld_tune_set(h, p, lanes * e, ch, ul, uc, e, il)
            res, det = L.ld_estimate_detail(h, p, n=a.n, tri=True)
            rel = abs(res.logdet - ref.logdet) / abs(ref.logdet)
            assert rel <= rtol_oracle, (lanes, ch, ul, uc, rel)
            assert abs(res.logdet - base) <= rtol_default * abs(base), (lanes, ch, e, ul, uc)
            np.testing.assert_array_equal(det["probe_steps"], np.array(ref.probe_steps))
            np.testing.assert_allclose(det["probe_K"], ref.probe_K,
                                       rtol=rtol_oracle * 100, atol=rtol_oracle * 100)
    finally:
        ctx.release(h)


def test_every_geometry_fp64(L, ctx):
    # 24 probes in FP64: 12 chunks per row; ragged n over the row chunks;
    # window 5, so the separate inner-product pass and a two-launch update
    # run with the forced update geometry as well
    _sweep(L, ctx, W.lap3d(17, 0.05), 24, L.LD_PREC_FP64, L.LD_VT_FP64, 1e-6, 1e-11, 2, 5)


def test_every_geometry_mixed(L, ctx):
    # 96 probes in FP32: 24 chunks per row (the default is L = 8, C = 3)
    _sweep(L, ctx, W.er_laplacian(6007, 40000, seed=4), 96, L.LD_PREC_MIXED, L.LD_VT_FP32,
           1e-4, 1e-5, 4, 2)


def test_entry_split_long_rows(L, ctx):
    # Wendland rows (~60 entries): every entry split of the product, FP64 and
    # FP16 vectors, against the oracle; fused inner product from the re-read
    # diagonal block row
    npr, s, m, k, seed = 32, 8, 20, 2, 4
    # FP16 vectors take a larger nugget (bound ratio 170; FP16 is refused on
    # nugget 1e-2, ratio ~1700)
    for prec, vec, tol, nug in ((L.LD_PREC_FP64, 2, 1e-6, 1e-2), (L.LD_PREC_HALF, 8, 1e-4, 0.1)):
        a = W.wendland(6000, 60.0, nug, seed=9)
        ref = oracle.oslq(a, npr, s, m, k, seed, lo_hint=nug)
        h = ctx.matrix(a, vt=L.LD_VT_FP32 if prec == L.LD_PREC_HALF else L.LD_VT_FP64,
                       lo_hint=nug)
        try:
            p = L.make_params(npr, s, m, k, seed, precision=prec)
            ncolv = npr // vec
            lanes = 1
            while lanes < ncolv:
                lanes *= 2
            base = None
            for e in _splits(lanes):
                _announce(f"entry split {e} n={a.n} nnz={a.nnz} prec={prec} L={lanes * e}")
                L.ld_tune_set(h, p, lanes * e, 1, lanes, 1, e)
                res = L.ld_estimate_ex(h, p)
                rel = abs(res.logdet - ref.logdet) / abs(ref.logdet)
                print(f"  rel {rel:.3e}", flush=True)
                assert rel <= tol, (e, rel)
                assert L.ld_estimate_ex(h, p).logdet == res.logdet
                if base is None:
                    base = res.logdet
                # a split changes the order of the FP32 row sums; with FP16
                # storage that moves the estimate within its rounding noise
                btol = 1e-12 if prec == L.LD_PREC_FP64 else 1e-4
                assert abs(res.logdet - base) <= btol * abs(base), e
        finally:
            ctx.release(h)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_row_tiles(L, ctx, prec):
    # the product taking its rows in tiles of 4 runs S rows apart: any valid
    # S gives the estimate up to the order of the FP64 partial sums; strides
    # with whole tiles only (n = 8000 = 20 tiles of 400) and with a ragged
    # remainder of rows in the plain order
    a = W.lap3d(20, 0.05)
    mixed = prec == "mixed"
    npr = 96 if mixed else 24
    P = L.LD_PREC_MIXED if mixed else L.LD_PREC_FP64
    vt = L.LD_VT_FP32 if mixed else L.LD_VT_FP64
    s, m, seed = 6, 14, 12
    tol, tight = (1e-4, 1e-5) if mixed else (1e-6, 1e-11)
    for k in (2, 5):
        ref = oracle.oslq(a, npr, s, m, k, seed)
        h = ctx.matrix(a, vt=vt)
        try:
            p = L.make_params(npr, s, m, k, seed, precision=P)
            base = L.ld_estimate_ex(h, p).logdet
            # (lanes, chunks, split, strides): rows per wave 64 / lanes
            geoms = ((8, 3, 1, (8, 24, 400, 2000)), (32, 2, 2, (2, 20, 22, 400))) if mixed else \
                    ((16, 1, 1, (4, 12, 20, 400)), (32, 1, 2, (2, 20, 22, 400)))
            for lanes, ch, e, strides in geoms:
                for S in strides:
                    for il in (0, 1):
                        _announce(f"row tiles n={a.n} prec={prec} k={k} L={lanes} C={ch} "
                                  f"split={e} interleave={il} stride={S}")
                        L.ld_tune_set(h, p, lanes, ch, 8, 3 if mixed else 2, e, il, S)
                        res, det = L.ld_estimate_detail(h, p, n=a.n, tri=True)
                        rel = abs(res.logdet - ref.logdet) / abs(ref.logdet)
                        assert rel <= tol, (lanes, S, il, rel)
                        assert abs(res.logdet - base) <= tight * abs(base), (lanes, S, il)
                        np.testing.assert_array_equal(det["probe_steps"],
                                                      np.array(ref.probe_steps))
                        assert L.ld_estimate_ex(h, p).logdet == res.logdet
            # a served request on the tiled geometry equals the same request alone
            L.ld_tune_set(h, p, geoms[0][0], geoms[0][1], 8, 3 if mixed else 2, 1, 1, 400)
            alone = L.ld_estimate_ex(h, p).logdet
            t = L.ld_submit(h, p)
            assert L.ld_wait(ctx.handle, t).logdet == alone
        finally:
            ctx.release(h)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_step_schedules(L, ctx, prec):
    # the two step schedules (the product subtracting the second-newest
    # window vector, or the update subtracting the whole window) give the
    # estimate up to rounding, for windows 2, 3, 5 and a window larger than
    # one launch of the update takes; served equals alone under either
    a = W.lap2d(45, 0.05)
    mixed = prec == "mixed"
    npr = 40 if mixed else 24
    P = L.LD_PREC_MIXED if mixed else L.LD_PREC_FP64
    vt = L.LD_VT_FP32 if mixed else L.LD_VT_FP64
    s, m, seed = 6, 16, 21
    tol, tight = (1e-4, 1e-5) if mixed else (1e-6, 1e-11)
    h = ctx.matrix(a, vt=vt)
    try:
        for k in (2, 3, 5, 10):
            ref = oracle.oslq(a, npr, s, m, k, seed)
            p = L.make_params(npr, s, m, k, seed, precision=P)
            vals = {}
            for ps in (1, 0):
                _announce(f"step schedule presub={ps} n={a.n} prec={prec} k={k}")
                L.ld_tune_set(h, p, 16, 1, 16, 1, 1, ps % 2, 0, ps)
                res, det = L.ld_estimate_detail(h, p, n=a.n, tri=True)
                rel = abs(res.logdet - ref.logdet) / abs(ref.logdet)
                assert rel <= tol, (k, ps, rel)
                np.testing.assert_array_equal(det["probe_steps"], np.array(ref.probe_steps))
                assert L.ld_estimate_ex(h, p).logdet == res.logdet
                t = L.ld_submit(h, p)
                assert L.ld_wait(ctx.handle, t).logdet == res.logdet
                vals[ps] = res.logdet
            assert abs(vals[0] - vals[1]) <= tight * abs(vals[1]), k
        with pytest.raises(L.LdError) as ei:
            L.ld_tune_set(h, L.make_params(npr, s, m, 2, seed, precision=P), 16, 1, 16, 1, 1, 0,
                          0, 2)
        assert ei.value.status == L.LD_E_INVALID_ARG
    finally:
        ctx.release(h)


def test_row_stride_rejected(L, ctx):
    a = W.lap2d(40, 0.1)
    h = ctx.matrix(a)
    try:
        p = L.make_params(24, 6, 10, 2, 1)  # FP64: 12 chunks per row
        base = L.ld_estimate_ex(h, p).logdet
        for lanes, ch, e, S in ((16, 1, 1, 6), (16, 1, 1, -4), (16, 1, 1, 32768),
                                (12, 1, 1, 16), (8, 2, 1, 4), (32, 1, 2, 3)):
            _announce(f"ld_tune_set rejects row stride {S} with L={lanes} C={ch} split={e}")
            with pytest.raises(L.LdError) as ei:
                L.ld_tune_set(h, p, lanes, ch, 16, 1, e, 0, S)
            assert ei.value.status == L.LD_E_INVALID_ARG
        assert L.ld_estimate_ex(h, p).logdet == base
    finally:
        ctx.release(h)


def test_invalid_geometry_rejected(L, ctx):
    a = W.lap2d(40, 0.1)
    h = ctx.matrix(a)
    try:
        p = L.make_params(24, 6, 10, 2, 1)
        base = L.ld_estimate_ex(h, p).logdet
        for bad in ((3, 3, 1), (0, 1, 1), (128, 1, 1), (4, 0, 1), (4, 5, 1), (1, 4, 1),
                    (2, 4, 1), (16, 1, 3), (16, 1, 16), (8, 2, 2), (64, 1, 8), (11, 1, 1),
                    (12, 1, 2), (24, 1, 2), (65, 1, 1)):
            _announce(f"ld_tune_set rejects L={bad[0]} C={bad[1]} split={bad[2]} "
                      "for 12 chunks per row")
            with pytest.raises(L.LdError) as ei:
                L.ld_tune_set(h, p, bad[0], bad[1], 4, 3, bad[2])
            assert ei.value.status == L.LD_E_INVALID_ARG
        _announce("ld_tune_set rejects an interleave flag other than 0 or 1")
        with pytest.raises(L.LdError) as ei:
            L.ld_tune_set(h, p, 16, 1, 16, 1, 1, 2)
        assert ei.value.status == L.LD_E_INVALID_ARG
        _announce("ld_tune_set rejects an update with L=11 C=1")
        with pytest.raises(L.LdError) as ei:
            L.ld_tune_set(h, p, 12, 1, 11, 1, 1)
        assert ei.value.status == L.LD_E_INVALID_ARG
        # nothing was stored: still the default geometry
        assert L.ld_estimate_ex(h, p).logdet == base
    finally:
        ctx.release(h)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_autotune_parity_and_reset(L, ctx, prec):
    a = W.lap3d(24, 0.02)
    mixed = prec == "mixed"
    npr = 64 if mixed else 32
    P = L.LD_PREC_MIXED if mixed else L.LD_PREC_FP64
    vt = L.LD_VT_FP32 if mixed else L.LD_VT_FP64
    s, m, k, seed = 8, 16, 2, 9
    ref = oracle.oslq(a, npr, s, m, k, seed)
    h = ctx.matrix(a, vt=vt)
    try:
        p = L.make_params(npr, s, m, k, seed, precision=P)
        untuned = L.ld_estimate_ex(h, p).logdet
        _announce(f"autotune n={a.n} probes={npr} prec={prec}")
        tr = L.ld_autotune(h, p, 5)
        print("  ", tr.as_dict(), flush=True)
        ncolv = npr // (4 if mixed else 2)
        assert tr.candidates >= 1
        assert tr.spmm_entry_split in (1, 2, 4, 8)
        # row tiles are tried at the grid's line and plane strides (24, 576)
        assert tr.spmm_row_stride in (0, 24, 576)
        assert tr.step_presub in (0, 1) and tr.step_presub_ms > 0 and tr.step_plain_ms > 0
        for lanes, ch in ((tr.spmm_lanes // tr.spmm_entry_split, tr.spmm_chunks),
                          (tr.update_lanes, tr.update_chunks)):
            assert (lanes, ch) in _usable(ncolv)
            assert 2 * (lanes * ch - ncolv) <= ncolv or tr.candidates == 1
        assert 0 < tr.spmm_ms <= tr.spmm_default_ms
        assert 0 < tr.update_ms <= tr.update_default_ms
        r1 = L.ld_estimate_ex(h, p).logdet
        r2 = L.ld_estimate_ex(h, p).logdet
        assert r1 == r2  # a fixed geometry stays bitwise reproducible
        tol = 1e-4 if mixed else 1e-6
        assert abs(r1 - ref.logdet) <= tol * abs(ref.logdet)
        assert abs(r1 - untuned) <= (1e-5 if mixed else 1e-11) * abs(untuned)
        _announce("autotune reset (reps = 0)")
        L.ld_autotune(h, p, 0)
        assert L.ld_estimate_ex(h, p).logdet == untuned
    finally:
        ctx.release(h)


def test_autotune_osa_iop(L, ctx):
    # OSA-IOP also tunes the sketch-run block (s columns)
    a = W.lap2d(70, 0.05)
    npr, s, m, k, seed = 40, 12, 14, 2, 5
    ref = oracle.osa_iop(a, npr, s, m, k, seed)
    h = ctx.matrix(a)
    try:
        p = L.make_params(npr, s, m, k, seed, method=L.LD_METHOD_OSA_IOP)
        _announce(f"autotune osa-iop n={a.n} probes={npr} s={s}")
        L.ld_autotune(h, p, 3)
        res = L.ld_estimate_ex(h, p)
        assert abs(res.logdet - ref.logdet) <= 1e-6 * abs(ref.logdet)
    finally:
        ctx.release(h)


def test_served_equals_alone_when_tuned(L):
    mats = [W.lap3d(20, 0.03), W.wendland(5000, 30.0, 0.02, seed=3)]
    reqs = []
    for i in range(len(mats)):
        for j, prec in enumerate((L.LD_PREC_FP64, L.LD_PREC_MIXED)):
            reqs.append((i, L.make_params(24 + 8 * j, 6, 12, 2, 70 + 3 * i + j, precision=prec)))
    c = L.Context(0)
    try:
        hs = [c.matrix(a) for a in mats]
        for i, p in reqs:
            L.ld_tune_set(hs[i], p, *((16, 1, 8, 2) if p.precision == L.LD_PREC_FP64
                                      else (16, 2, 32, 1)))
        _announce("served vs alone on tuned matrices")
        alone = [L.ld_estimate_ex(hs[i], p).logdet for i, p in reqs]
        tickets = [L.ld_submit(hs[i], p) for i, p in reqs]
        served = [L.ld_wait(c.handle, t).logdet for t in tickets]
        assert served == alone
    finally:
        c.close()

