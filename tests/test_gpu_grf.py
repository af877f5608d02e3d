"""GRF likelihood sweep (Section 4) on the GPU against the CPU oracle.

A Wendland C2 covariance Q(theta) on a small grid for several theta (support
radius theta / 10 grid spacings, nugget 1e-2 as the spectral lower bound),
a seeded smooth field x; every log-determinant (OSLQ and OSA-IOP, FP64)
within 1e-6 of the oracle, x^T Q x within 1e-12, L(theta) assembled alike,
and the swept requests (in flight together) equal to the same requests run
alone.  The paper's values need its field and theta units and are not
reproduced (parity unpinned for those).
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    from paper_2606_07004_amd import liblogdet
    liblogdet.lib()
    return liblogdet


def _mat(theta, ny=24, nx=30):
    return W.wendland_grid(ny, nx, W.grf_rho(theta), nugget=1e-2)


@pytest.mark.parametrize("method", ["oslq", "osa_iop"])
def test_grf_sweep_matches_oracle(L, method):
    from paper_2606_07004_amd import grf
    print(f"\n[case] grf sweep {method} 24x30 thetas 20,40,60", flush=True)
    thetas = (20, 40, 60)
    x = W.grf_field(24, 30, seed=7)
    if method == "oslq":
        p = L.make_params(30, 10, 40, 2, 1, method=L.LD_METHOD_OSLQ)
    else:
        p = L.make_params(21, 7, 20, 2, 1, method=L.LD_METHOD_OSA_IOP, tol=1e-6)
    with L.Context(0, max_slots=4) as c:
        recs = grf.theta_sweep(c, thetas, _mat, x, p, lo_hint=lambda th: 1e-2)
        alone = []
        for th in thetas:
            h = c.matrix(_mat(th), lo_hint=1e-2)
            alone.append(L.ld_estimate_ex(h, p).logdet)
            c.release(h)
    for rec, th, al in zip(recs, thetas, alone):
        a = _mat(th)
        if method == "oslq":
            ref = oracle.oslq(a, 30, 10, 40, 2, 1, lo_hint=1e-2)
        else:
            ref = oracle.osa_iop(a, 21, 7, 20, 2, 1, lo_hint=1e-2, tol=1e-6)
        q = sp.csr_matrix((a.values, a.col_idx, a.row_ptr), shape=(a.n, a.n))
        quad = float(x @ (q @ x))
        ll = 0.5 * ref.logdet - 0.5 * quad - 0.5 * a.n * math.log(2 * math.pi)
        rel = abs(rec["logdet"] - ref.logdet) / abs(ref.logdet)
        print(f"  theta {th}: logdet {rec['logdet']:.10g} oracle {ref.logdet:.10g} rel {rel:.2e} "
              f"loglik {rec['loglik']:.8g}", flush=True)
        assert rel <= 1e-6
        assert rec["quad"] == pytest.approx(quad, rel=1e-12)
        assert rec["loglik"] == pytest.approx(ll, rel=1e-6, abs=1e-6 * abs(ref.logdet))
        assert rec["logdet"] == al  # batched sweep == alone, bitwise


def test_quad_form_ragged(L):
    print("\n[case] quad form ragged n", flush=True)
    a = W.er_laplacian(5003, 20000, seed=9)
    x = np.random.default_rng(2).standard_normal(a.n)
    q = sp.csr_matrix((a.values, a.col_idx, a.row_ptr), shape=(a.n, a.n))
    with L.Context(0) as c:
        h = c.matrix(a)
        got = L.ld_quad_form(h, x)
        c.release(h)
    assert got == pytest.approx(float(x @ (q @ x)), rel=1e-12)
