"""Serving with continuous batching: ld_submit / ld_poll / ld_wait.

Each request's result must not depend on the other requests in flight: the
served result is compared bitwise with the same request run alone through
the blocking path, under both a roomy and a tiny HBM budget (one resident
request at a time), with requests of uneven size and both methods.
"""
import time

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    from paper_2606_07004_amd import liblogdet
    liblogdet.lib()
    return liblogdet


def _requests(L):
    mats = [W.lap2d(60, 0.05), W.lap3d(22, 1e-2), W.wendland(4000, 30.0, 0.02, seed=5),
            W.lap2d(90, 0.3), W.er_laplacian(8000, 64000, seed=2)]
    reqs = []
    for i, a in enumerate(mats):
        for method in (L.LD_METHOD_OSLQ, L.LD_METHOD_OSA_IOP):
            prec = L.LD_PREC_MIXED if (i + method) % 2 else L.LD_PREC_FP64
            reqs.append((i, L.make_params(18, 6, 12 + 3 * i, 2 + (i % 2), 100 + i,
                                          method=method, precision=prec)))
    return mats, reqs


def _alone(L, mats, reqs, vt=0):
    out = []
    with L.Context(0) as c:
        hs = [c.matrix(a, vt=vt) for a in mats]
        for i, p in reqs:
            out.append(L.ld_estimate_ex(hs[i], p).logdet)
    return out


def _served(L, mats, reqs, budget=0, slots=0, vt=0):
    c = L.Context(0, max_slots=slots, hbm_budget_bytes=budget)
    try:
        hs = [c.matrix(a, vt=vt) for a in mats]
        tickets = [L.ld_submit(hs[i], p) for i, p in reqs]
        res = [L.ld_wait(c.handle, t) for t in tickets]
        for h in hs:
            c.release(h)
    finally:
        c.close()
    return res


def test_served_equals_alone(L):
    print("\n[case] serving: 10 uneven requests, default budget", flush=True)
    mats, reqs = _requests(L)
    ref = _alone(L, mats, reqs)
    got = _served(L, mats, reqs)
    for r, g in zip(ref, got):
        assert g.logdet == r  # bitwise: private state, same kernels and geometry
        assert g.latency_ms > 0


def test_served_under_tiny_budget(L):
    print("\n[case] serving: budget for one resident request", flush=True)
    mats, reqs = _requests(L)
    ref = _alone(L, mats, reqs)
    # about 60 MB: the largest request here needs ~40 MB, so requests queue
    got = _served(L, mats, reqs, budget=60 << 20, slots=4)
    for r, g in zip(ref, got):
        assert g.logdet == r


def test_served_fp32_values(L):
    """Matrices with an FP32 copy of their values (the served form): FP32-
    vector requests read the FP32 values, FP64 ones the FP64 values."""
    print("\n[case] serving: FP32 value copies, mixed / auto / FP64 requests", flush=True)
    mats, base = _requests(L)
    precs = (L.LD_PREC_MIXED, L.LD_PREC_AUTO, L.LD_PREC_FP64)
    reqs = []
    for j, (i, p) in enumerate(base):
        q = L.make_params(p.n_probes, p.sketch_rank, p.krylov_steps, p.iop_window, p.seed,
                          method=p.method, precision=precs[j % 3])
        reqs.append((i, q))
    ref = _alone(L, mats, reqs, vt=L.LD_VT_FP32)
    got = _served(L, mats, reqs, vt=L.LD_VT_FP32)
    for r, g in zip(ref, got):
        assert g.logdet == r
    # the same requests in FP64 on FP64-only storage
    f64 = [(i, L.make_params(p.n_probes, p.sketch_rank, p.krylov_steps, p.iop_window, p.seed,
                             method=p.method, precision=L.LD_PREC_FP64)) for i, p in reqs]
    exact = _alone(L, mats, f64)
    for (i, p), g, e in zip(reqs, got, exact):
        if p.precision == L.LD_PREC_FP64:
            assert g.logdet == e
        else:
            assert abs(g.logdet - e) <= 1e-4 * abs(e), (i, p.precision, g.logdet, e)


def test_poll_semantics_and_errors(L):
    print("\n[case] serving: poll / wait / errors", flush=True)
    a = W.lap2d(120, 0.1)
    c = L.Context(0, hbm_budget_bytes=64 << 20)
    try:
        h = c.matrix(a)
        p = L.make_params(20, 6, 30, 2, 1)
        t = L.ld_submit(h, p)
        seen_pending = False
        res = None
        deadline = time.time() + 60
        while res is None and time.time() < deadline:
            res = L.ld_poll(c.handle, t)
            if res is None:
                seen_pending = True
                time.sleep(0.001)
        assert res is not None and np.isfinite(res.logdet)
        # a ticket is retired once its result was returned
        with pytest.raises(L.LdError) as e:
            L.ld_poll(c.handle, t)
        assert e.value.status == L.LD_E_UNKNOWN_TICKET
        with pytest.raises(L.LdError) as e:
            L.ld_wait(c.handle, 987654321)
        assert e.value.status == L.LD_E_UNKNOWN_TICKET
        # a request that can never fit the budget is refused at submit
        big = W.lap3d(60, 0.1)
        hb = c.matrix(big)
        with pytest.raises(L.LdError) as e:
            L.ld_submit(hb, L.make_params(120, 40, 80, 8, 0))
        assert e.value.status == L.LD_E_NO_MEMORY
        # a matrix with requests in flight cannot be destroyed
        t2 = L.ld_submit(h, p)
        try:
            with pytest.raises(L.LdError) as e:
                L.ld_destroy(h)
            assert e.value.status == L.LD_E_BUSY
        except AssertionError:
            raise
        finally:
            L.ld_wait(c.handle, t2)
        c.release(hb)
        c.release(h)
        print(f"  pending observed before completion: {seen_pending}")
    finally:
        c.close()


def test_serving_many_small_requests_throughput(L):
    print("\n[case] serving: 40 small requests vs sequential", flush=True)
    mats = [W.lap2d(100 + 5 * i, 0.01 * (i + 1)) for i in range(8)]
    with L.Context(0, max_slots=8) as c:
        hs = [c.matrix(a) for a in mats]
        ps = [L.make_params(30, 10, 25, 2, i, precision=L.LD_PREC_MIXED) for i in range(40)]
        t0 = time.perf_counter()
        seq = [L.ld_estimate_ex(hs[i % 8], p).logdet for i, p in enumerate(ps)]
        t_seq = time.perf_counter() - t0
        t0 = time.perf_counter()
        tk = [L.ld_submit(hs[i % 8], p) for i, p in enumerate(ps)]
        got = [L.ld_wait(c.handle, t).logdet for t in tk]
        t_srv = time.perf_counter() - t0
    assert got == seq
    print(f"  sequential {40 / t_seq:.1f} logdets/s, served {40 / t_srv:.1f} logdets/s")


def test_budget_charges_idle_slot_buffers(L):
    # A budget that holds about two of the large requests (or one large and
    # several small ones).  Idle slots keep their buffers for reuse, so the
    # ledger charges them too: the bytes the slot buffers hold never pass the
    # budget (idle buffers are released before a slot grows), no admitted
    # request fails to allocate, and every result equals the request alone.
    print("\n[case] serving: ledger with idle slot buffers", flush=True)
    small = W.lap2d(40, 0.2)
    large = W.lap3d(40, 0.05)
    with L.Context(0) as c0:
        hs, hl = c0.matrix(small), c0.matrix(large)
        ps = L.make_params(12, 4, 10, 2, 1)
        pl = L.make_params(40, 12, 20, 2, 2)
        b_small, b_large = L.ld_request_bytes(hs, ps), L.ld_request_bytes(hl, pl)
    assert b_large > 20 * b_small
    budget = int(2.2 * b_large)
    reqs = []
    for i in range(16):
        big = i % 3 == 1
        reqs.append((1 if big else 0,
                     L.make_params(40 if big else 12, 12 if big else 4, 20 if big else 10, 2,
                                   50 + i)))
    mats = [small, large]
    ref = _alone(L, mats, reqs)
    c = L.Context(0, max_slots=6, hbm_budget_bytes=budget)
    try:
        hm = [c.matrix(a) for a in mats]
        tickets = [L.ld_submit(hm[i], p) for i, p in reqs]
        got = [L.ld_wait(c.handle, t) for t in tickets]
        st = L.ld_serving_stats_get(c.handle)
        print(f"  budget {budget} peak held {st.peak_held_bytes} allocs {st.buffer_allocs} "
              f"frees {st.buffer_frees} peak active {st.peak_active}", flush=True)
        assert st.budget_bytes == budget
        assert st.peak_held_bytes <= budget
        assert st.completed == len(reqs)
        assert [g.logdet for g in got] == ref  # no LD_E_NO_MEMORY, same results
        for h in hm:
            c.release(h)
    finally:
        c.close()
