"""CPU checks of the C ABI boundary: the library is built, loads, and exports
every function include/liblogdet.h declares; host-side helpers compile and
agree with reference linear algebra.  No GPU calls."""
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "liblogdet.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:ld_status|const char\*)\s+(ld_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("ld_ctx_create", "ld_create_csr", "ld_estimate", "ld_estimate_ex",
                     "ld_submit", "ld_poll", "ld_wait", "ld_destroy", "ld_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2606_07004_amd import liblogdet as L
    handle = L.lib()
    for name in _declared():
        assert hasattr(handle, name), name
    bound = {n for n, _, _ in L._SIGNATURES}
    assert bound == set(_declared())
    nm = shutil.which("nm")
    if nm:
        out = subprocess.run([nm, "-D", "--defined-only", L.LIB_PATH], capture_output=True,
                             text=True).stdout
        exported = set(re.findall(r" T (ld_\w+)", out))
        assert set(_declared()) <= exported


def test_struct_layouts_match_header(tmp_path):
    # every field offset and size of the ctypes mirrors equals what a C
    # compiler makes of include/liblogdet.h
    from paper_2606_07004_amd import liblogdet as L
    import ctypes as C
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    exe = tmp_path / "abi_layout"
    subprocess.run([gcc, "-std=c99", "-I" + os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "csrc", "abi_layout.c"), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    mirrors = {"ld_ctx_opts": L.ld_ctx_opts, "ld_params": L.ld_params, "ld_result": L.ld_result,
               "ld_detail": L.ld_detail, "ld_tune_result": L.ld_tune_result,
               "ld_serving_stats": L.ld_serving_stats, "ld_graph_stats": L.ld_graph_stats}
    seen = {k: set() for k in mirrors}
    for line in out.strip().splitlines():
        struct, field, off, size = line.split()
        cls = mirrors[struct]
        if field == "-":
            assert C.sizeof(cls) == int(off), struct
            continue
        desc = getattr(cls, field)
        assert (desc.offset, desc.size) == (int(off), int(size)), (struct, field)
        seen[struct].add(field)
    for struct, cls in mirrors.items():
        assert seen[struct] == {name for name, _ in cls._fields_}, struct


@pytest.fixture(scope="module")
def gw_host(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = tmp_path_factory.mktemp("gw") / "gw_host"
    src = os.path.join(ROOT, "tests", "csrc", "gw_host.cpp")
    inc = os.path.join(ROOT, "paper_2606_07004_amd", "csrc")
    subprocess.run([gxx, "-O2", "-std=c++17", "-I" + inc, src, "-o", str(out)], check=True)
    return str(out)


def _run_gw(exe, d, e):
    inp = f"{len(d)}\n" + " ".join("%.17g" % x for x in d) + "\n" + \
        " ".join("%.17g" % x for x in e) + "\n"
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    lines = out.strip().split("\n")
    rc, bad, k = lines[0].split()
    pairs = np.array([[float(x) for x in ln.split()] for ln in lines[1:]])
    return int(rc), int(bad), float(k), pairs


def test_golub_welsch_host_build_matches_eigh(gw_host):
    rng = np.random.default_rng(0)
    for trial in range(120):
        n = int(rng.integers(1, 65))
        d = rng.uniform(0.05, 2.0, n)
        e = rng.uniform(-0.5, 0.5, n - 1)
        if trial % 5 == 0 and n > 2:
            e[int(rng.integers(0, n - 1))] = 0.0          # split matrix
        if trial % 7 == 0:
            d[:] = 1.0                                    # clustered spectrum
        rc, bad, k, pairs = _run_gw(gw_host, d, e)
        t = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
        lam, u = np.linalg.eigh(t)
        assert rc == 0
        np.testing.assert_allclose(np.sort(pairs[:, 0]), lam, atol=1e-13)
        # the quadrature rule (nodes, weights) must reproduce the moments
        for p in range(2 * n):
            lhs = np.sum(pairs[:, 1] ** 2 * pairs[:, 0] ** p)
            rhs = np.linalg.matrix_power(t, p)[0, 0]
            assert lhs == pytest.approx(rhs, rel=1e-10, abs=1e-12)
        if lam.min() > 0:
            assert bad == 0
            assert k == pytest.approx(float(np.sum(u[0] ** 2 * np.log(lam))), abs=1e-13)
        else:
            assert bad == 1


def test_golub_welsch_legendre_nodes(gw_host):
    for m in (3, 10, 40):
        j = np.arange(1, m)
        beta = j / np.sqrt(4.0 * j * j - 1.0)
        rc, bad, k, pairs = _run_gw(gw_host, np.zeros(m), beta)
        x, w = np.polynomial.legendre.leggauss(m)
        order = np.argsort(pairs[:, 0])
        np.testing.assert_allclose(pairs[order, 0], x, atol=1e-14)
        np.testing.assert_allclose(2 * pairs[order, 1] ** 2, w, atol=1e-14)
