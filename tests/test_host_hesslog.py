"""CPU tests of the Hessenberg-log routine the OSA-IOP kernel runs per Krylov
run (log(H) e1 by inverse scaling and squaring with a Gauss-Legendre Pade
step, Alg 1's log of the small Hessenberg matrix).  The header is compiled
for the host with g++ and driven through tests/csrc/hesslog_host.cpp.

Pins, each independent of the routine's own arithmetic:
  * scipy.linalg.logm on the Hessenberg matrices a truncated (window k)
    Arnoldi process produces for SPD operators (nonsymmetric, spectrum in the
    right half plane), and on symmetric tridiagonal ones;
  * the integral representation log(H) = int_0^inf [(1 + t)^-1 I - (t I + H)^-1] dt,
    evaluated by adaptive quadrature;
  * closed forms: diagonal H, H = c I, log(c H) e1 = log(H) e1 + log(c) e1,
    and the symmetric case through the eigendecomposition.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.integrate as si
import scipy.linalg as sl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = tmp_path_factory.mktemp("hesslog") / "hesslog_host"
    src = os.path.join(ROOT, "tests", "csrc", "hesslog_host.cpp")
    inc = os.path.join(ROOT, "paper_2606_07004_amd", "csrc")
    subprocess.run([gxx, "-O2", "-std=c++17", "-I" + inc, src, "-o", str(out)], check=True)
    return str(out)


def _log_e1(exe, H):
    n = H.shape[0]
    inp = f"{n}\n" + "\n".join(" ".join("%.17g" % x for x in row) for row in H) + "\n"
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    lines = out.strip().split("\n")
    return int(lines[0]), np.array([float(x) for x in lines[1:]])


def _iop_hessenberg(rng, n, m, k):
    """H (m x m) of m steps of Arnoldi with orthogonalisation against the k
    newest basis vectors only (the incomplete orthogonalisation of the OSA-IOP
    runs), on a random SPD matrix with eigenvalues in [0.05, 20]."""
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = (q * rng.uniform(0.05, 20.0, n)) @ q.T
    V = np.zeros((n, m + 1))
    H = np.zeros((m + 1, m))
    v = rng.standard_normal(n)
    V[:, 0] = v / np.linalg.norm(v)
    for t in range(m):
        w = A @ V[:, t]
        for i in range(max(0, t - k + 1), t + 1):
            H[i, t] = V[:, i] @ w
            w = w - H[i, t] * V[:, i]
        H[t + 1, t] = np.linalg.norm(w)
        V[:, t + 1] = w / H[t + 1, t]
    return H[:m, :m]


def test_matches_logm_on_iop_hessenberg(exe):
    rng = np.random.default_rng(1)
    for trial in range(24):
        m = int(rng.integers(2, 41))
        k = int(rng.integers(1, 5))
        H = _iop_hessenberg(rng, 80, m, k)
        rc, ell = _log_e1(exe, H)
        assert rc == 0
        ref = np.real(sl.logm(H))[:, 0]
        np.testing.assert_allclose(ell, ref, rtol=0, atol=1e-12 * max(1.0, np.abs(ref).max()))


def test_matches_integral_representation(exe):
    rng = np.random.default_rng(2)
    for m, k in ((6, 2), (12, 3), (20, 1)):
        H = _iop_hessenberg(rng, 50, m, k)
        rc, ell = _log_e1(exe, H)
        assert rc == 0
        e1 = np.zeros(m)
        e1[0] = 1.0
        eye = np.eye(m)

        # t in [0, inf) mapped to s in [0, 1): t = s / (1 - s), dt = ds / (1 - s)^2
        def f(s):
            t = s / (1.0 - s)
            return (e1 / (1.0 + t) - np.linalg.solve(t * eye + H, e1)) / (1.0 - s) ** 2
        ref, err = si.quad_vec(f, 0.0, 1.0, epsabs=1e-13, epsrel=1e-12, limit=2000)
        np.testing.assert_allclose(ell, ref, rtol=0, atol=1e-9)


def test_symmetric_tridiagonal_against_eigendecomposition(exe):
    rng = np.random.default_rng(3)
    for m in (1, 2, 5, 17, 48):
        d = rng.uniform(0.1, 30.0, m)
        e = rng.uniform(-3.0, 3.0, m - 1)
        T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
        lam, u = np.linalg.eigh(T)
        if lam.min() <= 0:
            T += (1e-2 - lam.min()) * np.eye(m)
            lam, u = np.linalg.eigh(T)
        rc, ell = _log_e1(exe, T)
        assert rc == 0
        ref = u @ (np.log(lam) * u[0])
        np.testing.assert_allclose(ell, ref, rtol=0, atol=1e-11 * max(1.0, np.abs(ref).max()))


def test_closed_forms(exe):
    # diagonal: log(H) e1 = log(h_11) e1
    H = np.diag([7.5, 0.2, 3.0, 40.0])
    rc, ell = _log_e1(exe, H)
    assert rc == 0
    np.testing.assert_allclose(ell, [np.log(7.5), 0, 0, 0], atol=1e-14)
    # a multiple of the identity, including 1 x 1
    for c in (1e-3, 1.0, 250.0):
        for m in (1, 6):
            rc, ell = _log_e1(exe, c * np.eye(m))
            assert rc == 0
            ref = np.zeros(m)
            ref[0] = np.log(c)
            np.testing.assert_allclose(ell, ref, atol=1e-13 * max(1.0, abs(np.log(c))))
    # log(c H) e1 = log(H) e1 + log(c) e1 (c > 0 commutes with H)
    rng = np.random.default_rng(4)
    H = _iop_hessenberg(rng, 40, 10, 2)
    _, a = _log_e1(exe, H)
    for c in (0.01, 37.0):
        _, b = _log_e1(exe, c * H)
        ref = a.copy()
        ref[0] += np.log(c)
        np.testing.assert_allclose(b, ref, rtol=0, atol=1e-10)
