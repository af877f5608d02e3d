"""Full-size GPU parity against stored oracle results.

The stored values (tests/golden/*.json) were written by
tests/golden/make_golden.py, which runs only the CPU FP64 oracle on the seeded
inputs; each file records the input's content digest, checked here before
comparing.  At these sizes the oracle takes minutes, so the comparison is
against the stored per-run values: every run's quadrature value, start norm
and Krylov dimension, then the assembled log-determinant (FP64 <= 1e-6,
FP32 or FP16 Krylov vectors <= 1e-4).
"""
import json
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

BUILDERS = {
    # the 128^3 grid: shifts 1e-3, 1e-2, 1e-1; windows 2, 4, 8; both methods
    "lap3d128_s1e-2_oslq_k2": lambda: W.lap3d(128, 1e-2),
    "lap3d128_s1e-3_oslq_k2": lambda: W.lap3d(128, 1e-3),
    "lap3d128_s1e-1_oslq_k2": lambda: W.lap3d(128, 1e-1),
    "lap3d128_s1e-2_oslq_k4": lambda: W.lap3d(128, 1e-2),
    "lap3d128_s1e-2_oslq_k8": lambda: W.lap3d(128, 1e-2),
    "lap3d128_s1e-2_osaiop_k2": lambda: W.lap3d(128, 1e-2),
    "lap3d128_s1e-1_osaiop_k2": lambda: W.lap3d(128, 1e-1),
    "lap3d128_s1e-2_osaiop_k4": lambda: W.lap3d(128, 1e-2),
    "lap3d128_s1e-2_osaiop_k8": lambda: W.lap3d(128, 1e-2),
    "er1e6_oslq_k4": lambda: W.er_laplacian(1_000_000, 8_000_000, seed=0, shift=0.05),
    "wendland5e5_oslq_k2": lambda: W.wendland(500_000, 48.0, 1e-2, seed=0),
    # values rounded to bfloat16: the matrix a BF16-valued product multiplies
    "wendland5e5_bf16_oslq_k2": lambda: W.round_values_bf16(W.wendland(500_000, 48.0, 1e-2,
                                                                       seed=0)),
}


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


def _load(name):
    with open(os.path.join(GOLDEN, name + ".json")) as f:
        return json.load(f)


def _run(L, ctx, name, precision, vt):
    gold = _load(name)
    print(f"\n[case] fullsize {name} precision={precision} vt={vt}", flush=True)
    a = BUILDERS[name]()
    assert W.csr_digest(a) == gold["digest"], "input differs from the one the oracle saw"
    method = L.LD_METHOD_OSLQ if gold["method"] == "oslq" else L.LD_METHOD_OSA_IOP
    h = ctx.matrix(a, vt=vt, lo_hint=gold["lo_hint"], hi_hint=gold["hi_hint"])
    try:
        p = L.make_params(gold["n_probes"], gold["sketch_rank"], gold["krylov_steps"],
                          gold["iop_window"], gold["seed"], method=method, precision=precision)
        res, det = L.ld_estimate_detail(h, p)
    finally:
        ctx.release(h)
    rel = abs(res.logdet - gold["logdet"]) / abs(gold["logdet"])
    print(f"  gpu {res.logdet!r} oracle {gold['logdet']!r} rel {rel:.3e} "
          f"device {res.device_ms:.1f} ms", flush=True)
    return gold, res, det, rel


OSLQ_CASES = [n for n in BUILDERS if "oslq" in n]
ALL_CASES = list(BUILDERS)


@pytest.mark.parametrize("name", ALL_CASES)
def test_fullsize_fp64_elementwise(L, ctx, name):
    gold, res, det, rel = _run(L, ctx, name, L.LD_PREC_FP64, L.LD_VT_FP64)
    assert rel <= 1e-6
    np.testing.assert_array_equal(det["probe_steps"], np.array(gold["probe_steps"]))
    np.testing.assert_allclose(det["probe_norm2"], gold["probe_norm2"], rtol=1e-10)
    np.testing.assert_allclose(det["probe_K"], gold["probe_K"], rtol=1e-7, atol=1e-9)
    assert res.shift_c == pytest.approx(gold["shift_c"], rel=1e-13)
    assert res.tr_sketch == pytest.approx(gold["tr_sketch"], rel=1e-9, abs=1e-6)
    assert res.tr_resid == pytest.approx(gold["tr_resid"], rel=1e-8)


@pytest.mark.parametrize("name", ALL_CASES)
def test_fullsize_mixed_within_1e4(L, ctx, name):
    gold, res, det, rel = _run(L, ctx, name, L.LD_PREC_MIXED, L.LD_VT_FP32)
    assert rel <= 1e-4


HALF_CASES = [n for n in BUILDERS if _load(n)["iop_window"] <= 4]


@pytest.mark.parametrize("name", HALF_CASES)
def test_fullsize_half(L, ctx, name):
    # FP16 Krylov vectors, FP32 values.  Accepted on spectral intervals with
    # lambda_hi <= 512 lambda_lo (windows up to 4), and then gated at 1e-4
    # like the FP32-vector precision; on wider intervals (the 128^3
    # Laplacian at shifts 1e-2 and 1e-3, the graph, the Wendland covariance)
    # the library refuses it
    gold = _load(name)
    ratio = gold["lambda_hi"] / gold["lambda_lo"]
    if ratio > 512:
        a = BUILDERS[name]()
        h = ctx.matrix(a, vt=L.LD_VT_FP32, lo_hint=gold["lo_hint"], hi_hint=gold["hi_hint"])
        try:
            method = L.LD_METHOD_OSLQ if gold["method"] == "oslq" else L.LD_METHOD_OSA_IOP
            p = L.make_params(gold["n_probes"], gold["sketch_rank"], gold["krylov_steps"],
                              gold["iop_window"], gold["seed"], method=method,
                              precision=L.LD_PREC_HALF)
            print(f"\n[case] fullsize {name} FP16 refused at bound ratio {ratio:.0f}", flush=True)
            with pytest.raises(L.LdError) as ei:
                L.ld_estimate_ex(h, p)
            assert ei.value.status == L.LD_E_INVALID_ARG
        finally:
            ctx.release(h)
        return
    gold, res, det, rel = _run(L, ctx, name, L.LD_PREC_HALF, L.LD_VT_FP32)
    assert rel <= 1e-4
    # OSLQ's sketch image is an FP64 product: start norms to rounding; OSA-IOP
    # builds its sketch from FP16 Krylov runs
    ntol = 1e-10 if gold["method"] == "oslq" else 1e-6
    np.testing.assert_allclose(det["probe_norm2"], gold["probe_norm2"], rtol=ntol)


def test_fullsize_bf16_values(L, ctx):
    # BF16 storage multiplies by the matrix with every value rounded to
    # bfloat16 (2^-9 relative): the reference is the FP64 oracle run on that
    # rounded matrix (tests/golden/wendland5e5_bf16_oslq_k2.json), and the
    # BF16-valued product with FP32 vectors is gated like the mixed precision
    gold, res, det, rel = _run(L, ctx, "wendland5e5_bf16_oslq_k2", L.LD_PREC_MIXED, L.LD_VT_BF16)
    assert rel <= 1e-4
    unrounded = _load("wendland5e5_oslq_k2")["logdet"]
    print(f"  rounding the values to bfloat16 moves the log-determinant by "
          f"{abs(gold['logdet'] - unrounded) / abs(unrounded):.3e}")
    np.testing.assert_allclose(det["probe_norm2"], gold["probe_norm2"], rtol=1e-6)


@pytest.mark.parametrize("prec_name", ["FP64", "MIXED"])
def test_fullsize_osa_iop_two_pass_sketch(L, ctx, prec_name):
    # the 128^3 Laplacian, OSA-IOP, window 2, with the memory-lean two-pass
    # sketch image: bitwise the kept-basis estimate, within the gate of the
    # stored oracle result, in a fraction of the device memory
    name = "lap3d128_s1e-2_osaiop_k2"
    gold = _load(name)
    a = BUILDERS[name]()
    assert W.csr_digest(a) == gold["digest"]
    prec = getattr(L, "LD_PREC_" + prec_name)
    vt = L.LD_VT_FP64 if prec_name == "FP64" else L.LD_VT_FP32
    print(f"\n[case] fullsize {name} two-pass sketch {prec_name}", flush=True)
    h = ctx.matrix(a, vt=vt)
    try:
        p1 = L.make_params(gold["n_probes"], gold["sketch_rank"], gold["krylov_steps"],
                           gold["iop_window"], gold["seed"], method=L.LD_METHOD_OSA_IOP,
                           precision=prec)
        p2 = L.make_params(gold["n_probes"], gold["sketch_rank"], gold["krylov_steps"],
                           gold["iop_window"], gold["seed"], method=L.LD_METHOD_OSA_IOP,
                           precision=prec, sketch_passes=2)
        b1, b2 = L.ld_request_bytes(h, p1), L.ld_request_bytes(h, p2)
        r2 = L.ld_estimate_ex(h, p2)
        r1 = L.ld_estimate_ex(h, p1)
    finally:
        ctx.release(h)
    rel = abs(r2.logdet - gold["logdet"]) / abs(gold["logdet"])
    print(f"  two-pass {r2.logdet!r} ({b2 / 1e9:.2f} GB, {r2.device_ms:.1f} ms) one-pass "
          f"{r1.logdet!r} ({b1 / 1e9:.2f} GB, {r1.device_ms:.1f} ms) rel {rel:.2e}", flush=True)
    assert r2.logdet == r1.logdet
    assert rel <= (1e-6 if prec_name == "FP64" else 1e-4)
    assert b2 < 0.4 * b1
