"""HIP-graph replay of blocking estimates.

The second blocking estimate of a context with the same matrix and the same
parameters apart from the seed is captured into a graph; later ones replay it.
A replay runs the same kernels in the same order on the same buffers, so every
result must be bitwise the one of a context that launches kernel by kernel
(graph mode 0), for every seed.  Replays are interleaved with other device
work (estimates of another shape, served requests, no-allocation estimates,
copy kernels, synchronisations) and each replay is checked, not only the
first.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    from paper_2606_07004_amd import liblogdet
    liblogdet.lib()  # fails loudly when the HIP library is missing
    return liblogdet


@pytest.fixture(scope="module")
def ctxs(L):
    eager = L.Context(0)
    L.ld_graph_mode(eager.handle, 0)
    graph = L.Context(0)
    yield eager, graph
    eager.close()
    graph.close()


def _announce(msg):
    print(f"\n[case] {msg}", flush=True)


CASES = {
    "oslq_mixed": dict(method="OSLQ", prec="MIXED", npr=40, s=12, m=20, k=2),
    "oslq_fp64_gauss": dict(method="OSLQ", prec="FP64", npr=24, s=8, m=15, k=3,
                            dist="GAUSSIAN"),
    "oslq_half": dict(method="OSLQ", prec="HALF", npr=32, s=8, m=15, k=2),
    "osa_iop_one_pass": dict(method="OSA_IOP", prec="MIXED", npr=24, s=8, m=12, k=2),
    "osa_iop_two_pass": dict(method="OSA_IOP", prec="FP64", npr=24, s=8, m=12, k=3, passes=2),
    "so_slq": dict(method="SO_SLQ", prec="MIXED", npr=30, s=16, m=12, k=2, sub=6),
    "slq_no_sketch": dict(method="OSLQ", prec="MIXED", npr=16, s=0, m=10, k=2),
}


def _params(L, c, seed):
    return L.make_params(c["npr"], c["s"], c["m"], c["k"], seed,
                         method=getattr(L, "LD_METHOD_" + c["method"]),
                         precision=getattr(L, "LD_PREC_" + c["prec"]),
                         probe_dist=getattr(L, "LD_PROBE_" + c.get("dist", "RADEMACHER")),
                         subspace_rank=c.get("sub", 0), sketch_passes=c.get("passes", 0))


def _same(r1, r2):
    for f in ("logdet", "tr_sketch", "tr_resid", "probe_steps", "min_steps", "n_breakdowns",
              "basis_rank", "matvecs"):
        assert getattr(r1, f) == getattr(r2, f), f


@pytest.mark.parametrize("name", sorted(CASES))
def test_replay_bitwise_equals_eager(L, ctxs, name):
    eager, graph = ctxs
    c = CASES[name]
    a = W.lap3d(18, 0.05)
    other = W.lap2d(50, 0.2)
    vt = L.LD_VT_FP64 if c["prec"] == "FP64" else L.LD_VT_FP32
    he, hg = eager.matrix(a, vt=vt), graph.matrix(a, vt=vt)
    ho = graph.matrix(other, vt=L.LD_VT_FP32)
    try:
        st0 = L.ld_graph_stats_get(graph.handle)
        for i, seed in enumerate([3, 3, 11, 12, 3, 99]):
            _announce(f"graph replay {name} {a.name} call {i} seed {seed}")
            ref = L.ld_estimate_ex(he, _params(L, c, seed))
            got = L.ld_estimate_ex(hg, _params(L, c, seed))
            _same(got, ref)
            assert np.isfinite(got.logdet)
            # other device work between replays: another shape on the same
            # context (its own graph after two calls), a served request, a
            # no-allocation estimate and a plain copy kernel on the stream
            L.ld_estimate_ex(ho, L.make_params(12, 4, 8, 2, 100 + i))
            t = L.ld_submit(ho, L.make_params(12, 4, 8, 2, 200 + i))
            L.ld_estimate_noalloc(ho, L.make_params(12, 4, 8, 2, 300 + i))
            L.ld_debug_copy(graph.handle, 1 << 22, 2)
            L.ld_wait(graph.handle, t)
        st1 = L.ld_graph_stats_get(graph.handle)
        # first call eager, second captured and replayed, the rest replayed
        # (the same for the other matrix, whose seed changes every call)
        assert st1.captures - st0.captures == 2
        assert st1.replays - st0.replays == 2 * (6 - 1)
    finally:
        eager.release(he)
        graph.release(hg)
        graph.release(ho)


def test_detail_after_replay(L, ctxs):
    eager, graph = ctxs
    a = W.lap2d(60, 0.1)
    c = CASES["osa_iop_one_pass"]
    he, hg = eager.matrix(a, vt=L.LD_VT_FP32), graph.matrix(a, vt=L.LD_VT_FP32)
    try:
        for seed in (5, 6, 7):
            _announce(f"graph replay detail {a.name} seed {seed}")
            re_, de = L.ld_estimate_detail(he, _params(L, c, seed), n=a.n, tri=True, basis=True)
            rg, dg = L.ld_estimate_detail(hg, _params(L, c, seed), n=a.n, tri=True, basis=True)
            _same(rg, re_)
            for k in de:
                np.testing.assert_array_equal(dg[k], de[k])
        assert L.ld_graph_stats_get(graph.handle).replays >= 1
    finally:
        eager.release(he)
        graph.release(hg)


def test_uncapturable_estimates_stay_eager(L, ctxs):
    _, graph = ctxs
    a = W.lap2d(40, 0.1)
    h = graph.matrix(a, vt=L.LD_VT_FP32)
    try:
        _announce("graph: adaptive and profiled estimates launch kernel by kernel")
        st0 = L.ld_graph_stats_get(graph.handle)
        for _ in range(3):
            L.ld_estimate_ex(h, L.make_params(16, 4, 30, 2, 1, adapt_tol=1e-6, adapt_every=5))
        L.ld_profile_enable(graph.handle, L.LD_PROF_ALL)
        try:
            for _ in range(3):
                L.ld_estimate_ex(h, L.make_params(16, 4, 12, 2, 1))
        finally:
            L.ld_profile_enable(graph.handle, 0)
        st1 = L.ld_graph_stats_get(graph.handle)
        assert st1.captures == st0.captures and st1.replays == st0.replays
        assert st1.eager - st0.eager == 6
    finally:
        graph.release(h)


def test_destroy_tune_and_workspace_growth_drop_graphs(L, ctxs):
    _, graph = ctxs
    a = W.lap2d(40, 0.1)
    h = graph.matrix(a, vt=L.LD_VT_FP32)
    p = L.make_params(16, 4, 12, 2, 1)
    _announce("graph: cache upkeep (tune change, workspace growth, destroy)")
    L.ld_estimate_ex(h, p)
    r = L.ld_estimate_ex(h, p)
    st = L.ld_graph_stats_get(graph.handle)
    assert st.cached >= 1
    cap0 = st.captures
    # a new geometry for the block (FP64: 8 lanes x 1 chunk cover the 16
    # columns): the old graph no longer matches, the next two calls run
    # eager and then captured
    L.ld_tune_set(h, p, 8, 1, 8, 1)
    L.ld_estimate_ex(h, p)
    assert L.ld_graph_stats_get(graph.handle).captures == cap0
    L.ld_estimate_ex(h, p)
    assert L.ld_graph_stats_get(graph.handle).captures == cap0 + 1
    # a request larger than the workspace: it grows and every graph goes
    big = W.lap3d(40, 0.1)
    hb = graph.matrix(big, vt=L.LD_VT_FP32)
    L.ld_estimate_ex(hb, L.make_params(64, 16, 30, 2, 1))
    assert L.ld_graph_stats_get(graph.handle).cached == 0
    graph.release(hb)
    # the same estimate again: eager once, then captured, bitwise as before
    L.ld_tune_set(h, p, 8, 1, 8, 1)
    r2 = L.ld_estimate_ex(h, p)
    r3 = L.ld_estimate_ex(h, p)
    assert r2.logdet == r3.logdet
    cached = L.ld_graph_stats_get(graph.handle).cached
    assert cached >= 1
    graph.release(h)
    assert L.ld_graph_stats_get(graph.handle).cached == cached - 1
    del r


def test_mode_switch(L):
    ctx = L.Context(0)
    try:
        a = W.lap2d(30, 0.3)
        h = ctx.matrix(a, vt=L.LD_VT_FP32)
        p = L.make_params(12, 4, 10, 2, 9)
        _announce("graph: mode 1 -> 0 drops the graphs, results unchanged")
        vals = [L.ld_estimate_ex(h, p).logdet for _ in range(3)]
        assert L.ld_graph_stats_get(ctx.handle).cached == 1
        L.ld_graph_mode(ctx.handle, 0)
        st = L.ld_graph_stats_get(ctx.handle)
        assert st.cached == 0 and st.mode == 0 and st.capture_failed == 0
        vals.append(L.ld_estimate_ex(h, p).logdet)
        assert len(set(vals)) == 1
        with pytest.raises(L.LdError):
            L.ld_graph_mode(ctx.handle, 2)
    finally:
        ctx.close()


def test_concurrent_callers_share_the_cache(L):
    # blocking estimates of one context from several host threads: they run
    # one at a time, capture and replay through one cache, and every result
    # is bitwise the kernel-by-kernel one
    import threading
    ctx = L.Context(0)
    ref_ctx = L.Context(0)
    L.ld_graph_mode(ref_ctx.handle, 0)
    try:
        mats = [W.lap2d(48, 0.1), W.lap3d(14, 0.2), W.lap2d(40, 0.05)]
        hs = [ctx.matrix(a, vt=L.LD_VT_FP32) for a in mats]
        hr = [ref_ctx.matrix(a, vt=L.LD_VT_FP32) for a in mats]
        jobs = [(i % 3, 500 + i) for i in range(24)]
        p = lambda seed: L.make_params(16, 4, 12, 2, seed, precision=L.LD_PREC_MIXED)
        _announce("graph: 4 threads x 6 estimates on one context")
        want = {j: L.ld_estimate_ex(hr[j[0]], p(j[1])).logdet for j in jobs}
        # one call per matrix first, the largest first, so that the workspace
        # does not grow (and drop the graphs) once the threads run
        for i in (1, 0, 2):
            L.ld_estimate_ex(hs[i], p(1))
        got = {}
        errs = []

        def worker(part):
            try:
                for j in part:
                    got[j] = L.ld_estimate_ex(hs[j[0]], p(j[1])).logdet
            except Exception as e:  # reported below
                errs.append(e)
        ths = [threading.Thread(target=worker, args=(jobs[t::4],)) for t in range(4)]
        for t in ths:
            t.start()
        for t in ths:
            t.join()
        assert not errs, errs
        assert got == want
        st = L.ld_graph_stats_get(ctx.handle)
        assert st.captures == 3 and st.replays == 24
    finally:
        ctx.close()
        ref_ctx.close()
