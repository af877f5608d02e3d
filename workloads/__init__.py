"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module builds sparse SPD matrices (CSR, FP64 values, int32 indices) and
request streams.  It holds none of the estimator's arithmetic: no Krylov
recurrence, no quadrature, no trace assembly.  The only "answers" here are
closed-form log-determinants of the Dirichlet Laplacians, computed from their
known eigenvalues, which the tests and the benchmark report beside estimates.

Matrix families stand in for the application classes of the paper's
experiments (Section 4, Table 1): stencil/FEM-like operators (2D and 3D
Laplacians), an unstructured graph (Erdos-Renyi graph Laplacian) and dense
local coupling (compactly supported Wendland C2 covariance, the kernel of the
paper's Gaussian-random-field experiment, Section 4, Tables 4-5).
"""
from __future__ import annotations

import dataclasses
import math
import os

import numpy as np
import scipy.sparse as sp

__all__ = [
    "Csr", "lap2d", "lap3d", "er_laplacian", "wendland", "diag_matrix",
    "random_spd_dense", "from_dense", "lap2d_exact_logdet",
    "lap3d_exact_logdet", "request_stream", "csr_digest", "round_values_bf16",
]


@dataclasses.dataclass
class Csr:
    """Compressed sparse row matrix: int32 row_ptr[n+1], int32 col_idx[nnz],
    float64 values[nnz]; column indices sorted and unique inside each row."""
    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    values: np.ndarray
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.values, self.col_idx, self.row_ptr),
                             shape=(self.n, self.n))

    def to_dense(self) -> np.ndarray:
        return self.to_scipy().toarray()


def _from_scipy(m: sp.spmatrix, name: str) -> Csr:
    m = sp.csr_matrix(m)
    m.sum_duplicates()
    m.sort_indices()
    return Csr(n=m.shape[0],
               row_ptr=np.ascontiguousarray(m.indptr, dtype=np.int32),
               col_idx=np.ascontiguousarray(m.indices, dtype=np.int32),
               values=np.ascontiguousarray(m.data, dtype=np.float64),
               name=name)


def from_dense(a: np.ndarray, name: str = "dense") -> Csr:
    """CSR of a dense matrix, keeping every entry that is not exactly zero."""
    return _from_scipy(sp.csr_matrix(np.asarray(a, dtype=np.float64)), name)


def _stencil(dims, shift: float, name: str) -> Csr:
    """Dirichlet Laplacian on a tensor grid with natural (first axis fastest)
    ordering: diagonal 2*len(dims) + shift, -1 to each grid neighbour.

    Built row-major straight into CSR: every row's candidate columns are
    its neighbours at offsets -stride_k .. +stride_k (ascending, so each row's
    columns come out sorted), kept where the neighbour lies on the grid."""
    dims = tuple(int(d) for d in dims)
    n = int(np.prod(dims))
    idx = np.arange(n, dtype=np.int64)
    strides = np.cumprod((1,) + dims[:-1]).astype(np.int64)
    offs, checks = [], []
    for k in reversed(range(len(dims))):      # -stride_last ... -1
        offs.append(-strides[k])
        checks.append((k, -1))
    offs.append(0)
    checks.append(None)
    for k in range(len(dims)):                # +1 ... +stride_last
        offs.append(strides[k])
        checks.append((k, 1))
    cand = np.empty((n, len(offs)), dtype=np.int64)
    valid = np.empty((n, len(offs)), dtype=bool)
    for j, (off, chk) in enumerate(zip(offs, checks)):
        cand[:, j] = idx + off
        if chk is None:
            valid[:, j] = True
        else:
            k, step = chk
            coord = (idx // strides[k]) % dims[k]
            valid[:, j] = (coord + step >= 0) & (coord + step < dims[k])
    counts = valid.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col_idx = cand[valid]
    vals = np.where(col_idx == np.repeat(idx, counts), 2.0 * len(dims) + shift, -1.0)
    return Csr(n=n, row_ptr=row_ptr.astype(np.int32), col_idx=col_idx.astype(np.int32),
               values=np.ascontiguousarray(vals, dtype=np.float64), name=name)


def lap2d(N: int, shift: float) -> Csr:
    """5-point Dirichlet Laplacian on an N x N grid plus shift*I, row i = x + N*y."""
    return _stencil((N, N), shift, f"lap2d_{N}_shift{shift:g}")


def lap3d(N: int, shift: float) -> Csr:
    """7-point Dirichlet Laplacian on an N^3 grid plus shift*I."""
    return _stencil((N, N, N), shift, f"lap3d_{N}_shift{shift:g}")


def _dirichlet_eigs_1d(N: int) -> np.ndarray:
    k = np.arange(1, N + 1, dtype=np.float64)
    return 2.0 - 2.0 * np.cos(np.pi * k / (N + 1))


def lap2d_exact_logdet(N: int, shift: float) -> float:
    """sum over i,j of log(4 - 2cos(pi i/(N+1)) - 2cos(pi j/(N+1)) + shift)."""
    e = _dirichlet_eigs_1d(N)
    lam = e[:, None] + e[None, :] + shift
    return math.fsum(np.log(lam).ravel())


def lap3d_exact_logdet(N: int, shift: float) -> float:
    """sum over i,j,k of log(6 - 2cos(.) - 2cos(.) - 2cos(.) + shift)."""
    e = _dirichlet_eigs_1d(N)
    total = []
    for a in e:  # one plane at a time keeps memory at N^2
        lam = a + e[:, None] + e[None, :] + shift
        total.append(math.fsum(np.log(lam).ravel()))
    return math.fsum(total)


def er_laplacian(n: int, n_edges: int, seed: int = 0, shift: float = 0.05,
                 wlo: float = 0.5, whi: float = 1.5) -> Csr:
    """Weighted Erdos-Renyi graph Laplacian plus shift*I.

    n_edges distinct undirected edges without self-loops are drawn uniformly
    with numpy's PCG64(seed); duplicates and loops are redrawn.  Weights are
    U(wlo, whi), drawn after the edge set is fixed, in sorted-edge order.
    Rows keep the natural (random) vertex order.  nnz = n + 2*n_edges.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    keys = np.empty(0, dtype=np.int64)
    while keys.size < n_edges:
        need = n_edges - keys.size
        u = rng.integers(0, n, size=need, dtype=np.int64)
        v = rng.integers(0, n, size=need, dtype=np.int64)
        ok = u != v
        lo = np.minimum(u[ok], v[ok])
        hi = np.maximum(u[ok], v[ok])
        keys = np.union1d(keys, lo * n + hi)
    lo = keys // n
    hi = keys % n
    w = rng.uniform(wlo, whi, size=n_edges)
    deg = np.bincount(lo, weights=w, minlength=n) + np.bincount(hi, weights=w, minlength=n)
    rows = np.concatenate([lo, hi, np.arange(n)])
    cols = np.concatenate([hi, lo, np.arange(n)])
    vals = np.concatenate([-w, -w, deg + shift])
    m = sp.coo_matrix((vals, (rows, cols)), shape=(n, n))
    return _from_scipy(m, f"er_{n}_{n_edges}_seed{seed}")


def _wendland_native(h, n, pts, cell_sorted, ncell, rho, scale, nugget, name) -> Csr:
    """The C helper's neighbour search over the 3 x 3 cells around each point
    (rows split over host threads); the same matrix as the NumPy path."""
    import ctypes as C
    from concurrent.futures import ThreadPoolExecutor
    cell_start = np.searchsorted(cell_sorted, np.arange(ncell * ncell + 1), side="left")
    cell_start = np.ascontiguousarray(cell_start, dtype=np.int64)
    cell_sorted = np.ascontiguousarray(cell_sorted, dtype=np.int64)
    dp, i64p, i32p = C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_int32)
    pp, cp, sp_ = pts.ctypes.data_as(dp), cell_sorted.ctypes.data_as(i64p), \
        cell_start.ctypes.data_as(i64p)
    nt = max(1, min(16, os.cpu_count() or 1, n // 65536))
    bounds = [(n * t // nt, n * (t + 1) // nt) for t in range(nt)]
    counts = np.zeros(n, dtype=np.int64)
    with ThreadPoolExecutor(nt) as ex:
        list(ex.map(lambda b: h.wendland_count(b[0], b[1], pp, cp, sp_, ncell, rho,
                                               counts.ctypes.data_as(i64p)), bounds))
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("wendland: nnz does not fit int32")
    col = np.empty(int(row_ptr[-1]), dtype=np.int32)
    val = np.empty(int(row_ptr[-1]), dtype=np.float64)
    with ThreadPoolExecutor(nt) as ex:
        list(ex.map(lambda b: h.wendland_fill(b[0], b[1], pp, cp, sp_, ncell, rho, scale, nugget,
                                              row_ptr.ctypes.data_as(i64p), col.ctypes.data_as(i32p),
                                              val.ctypes.data_as(dp)), bounds))
    return Csr(n=n, row_ptr=row_ptr.astype(np.int32), col_idx=col, values=val, name=name)


def wendland(n: int, nnz_per_row: float = 48.0, nugget: float = 1e-2,
             seed: int = 0, scale: float = 1.0, use_native: bool = True) -> Csr:
    """Wendland C2 covariance matrix on n uniform points in [0,1]^2.

    phi(r) = (1 - r/rho)^4_+ (4 r/rho + 1) with support radius
    rho = sqrt(nnz_per_row / (pi n)), so an interior row holds about
    nnz_per_row off-diagonal entries; diagonal = scale*phi(0) + nugget.
    Points (PCG64(seed)) are sorted by rho-cell, row-major over cells, so that
    neighbouring rows are neighbouring points.  With the C helper built
    (workloads.native) the neighbour search runs there, giving bitwise the
    matrix of the NumPy path (use_native=False).
    """
    from scipy.spatial import cKDTree
    rng = np.random.Generator(np.random.PCG64(seed))
    pts = rng.random((n, 2))
    rho = math.sqrt(nnz_per_row / (math.pi * n))
    ncell = max(1, int(math.floor(1.0 / rho)))
    cx = np.minimum((pts[:, 0] * ncell).astype(np.int64), ncell - 1)
    cy = np.minimum((pts[:, 1] * ncell).astype(np.int64), ncell - 1)
    cell = cy * ncell + cx
    order = np.argsort(cell, kind="stable")
    pts = np.ascontiguousarray(pts[order])
    name = f"wendland_{n}_nugget{nugget:g}_seed{seed}"
    from . import native
    h = native.lib() if use_native else None
    if h is not None:
        return _wendland_native(h, n, pts, np.ascontiguousarray(cell[order]), ncell, rho, scale,
                                nugget, name)
    tree = cKDTree(pts)
    pairs = tree.query_pairs(rho, output_type="ndarray").astype(np.int64)
    d = pts[pairs[:, 0]] - pts[pairs[:, 1]]
    r = np.sqrt(d[:, 0] ** 2 + d[:, 1] ** 2) / rho
    keep = r < 1.0
    pairs, r = pairs[keep], r[keep]
    # (1 - r)^4 as two squarings: only correctly rounded basic operations, so
    # the values do not depend on the host's vectorised pow (and match the C
    # helper's bit for bit)
    t = 1.0 - r
    t2 = t * t
    phi = scale * (t2 * t2) * (4.0 * r + 1.0)
    rows = np.concatenate([pairs[:, 0], pairs[:, 1], np.arange(n)])
    cols = np.concatenate([pairs[:, 1], pairs[:, 0], np.arange(n)])
    vals = np.concatenate([phi, phi, np.full(n, scale + nugget)])
    m = sp.coo_matrix((vals, (rows, cols)), shape=(n, n))
    return _from_scipy(m, name)


def wendland_grid(ny: int, nx: int, rho: float, nugget: float = 1e-2, scale: float = 1.0) -> Csr:
    """Wendland C2 covariance matrix on the ny x nx unit-spaced grid.

    Grid point (iy, ix) is row iy * nx + ix; the entry between points at
    distance r < rho is scale * phi(r) with phi(r) = (1 - r/rho)^4 (4 r/rho + 1),
    the diagonal scale + nugget.  On a grid every interior row holds the same
    stencil of about pi rho^2 entries; columns are sorted within a row.
    """
    n = ny * nx
    R = int(math.ceil(rho))
    offs = [(dy, dx) for dy in range(-R, R + 1) for dx in range(-R, R + 1)
            if dy * dy + dx * dx < rho * rho]
    iy = np.repeat(np.arange(ny, dtype=np.int64), nx)
    ix = np.tile(np.arange(nx, dtype=np.int64), ny)
    noff = len(offs)
    cols = np.empty((n, noff), dtype=np.int64)
    vals = np.empty(noff, dtype=np.float64)
    for j, (dy, dx) in enumerate(offs):  # (dy, dx) ascending: columns ascending
        ok = (iy + dy >= 0) & (iy + dy < ny) & (ix + dx >= 0) & (ix + dx < nx)
        c = (iy + dy) * nx + (ix + dx)
        c[~ok] = -1
        cols[:, j] = c
        r = math.sqrt(dy * dy + dx * dx) / rho
        vals[j] = scale * (1.0 - r) ** 4 * (4.0 * r + 1.0) + (nugget if (dy, dx) == (0, 0) else 0.0)
    valid = cols >= 0
    counts = valid.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("wendland_grid: nnz does not fit int32")
    col_idx = cols[valid].astype(np.int32)
    values = np.broadcast_to(vals, (n, noff))[valid].copy()
    del cols, valid
    return Csr(n=n, row_ptr=row_ptr.astype(np.int32), col_idx=col_idx, values=values,
               name=f"wendland_grid_{ny}x{nx}_rho{rho:g}_nugget{nugget:g}")


def grf_field(ny: int, nx: int, seed: int = 0, waves: int = 16) -> np.ndarray:
    """Seeded smooth synthetic field on the grid (row-major, unit variance):
    a sum of plane waves with wavelengths between 10 and 200 grid cells and
    random phases, plus white noise of standard deviation 0.1 (PCG64(seed))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    iy = np.repeat(np.arange(ny, dtype=np.float64), nx)
    ix = np.tile(np.arange(nx, dtype=np.float64), ny)
    x = np.zeros(ny * nx)
    for _ in range(waves):
        lam = math.exp(rng.uniform(math.log(10.0), math.log(200.0)))
        ang = rng.uniform(0.0, math.pi)
        ph = rng.uniform(0.0, 2 * math.pi)
        k = 2 * math.pi / lam
        x += rng.standard_normal() * np.cos(k * (math.cos(ang) * ix + math.sin(ang) * iy) + ph)
    x /= max(float(np.std(x)), 1e-300)
    return x + 0.1 * rng.standard_normal(ny * nx)


# GRF likelihood sweep (Section 4): candidate parameters and the support
# radius of each on the unit-spaced grid.  The paper does not state the
# units of theta; here rho = theta / 10 grid spacings.
GRF_THETAS = (20, 30, 40, 50, 60, 70, 80)


def grf_rho(theta: float) -> float:
    return theta / 10.0


def diag_matrix(values) -> Csr:
    """Diagonal matrix (breakdown cases: d distinct values stop a Krylov run
    after d steps)."""
    v = np.asarray(values, dtype=np.float64)
    n = v.size
    return Csr(n=n, row_ptr=np.arange(n + 1, dtype=np.int32),
               col_idx=np.arange(n, dtype=np.int32), values=v.copy(),
               name=f"diag_{n}")


def random_spd_dense(n: int, seed: int, lo: float = 0.1, hi: float = 10.0) -> np.ndarray:
    """Dense SPD matrix Q = U diag(lam) U^T with log-uniform lam in [lo, hi]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.exp(rng.uniform(math.log(lo), math.log(hi), size=n))
    q = (u * lam) @ u.T
    return 0.5 * (q + q.T)


def round_values_bf16(a: Csr) -> Csr:
    """The same matrix with every value rounded once to bfloat16 (8 exponent
    bits, 7 stored mantissa bits), round-to-nearest, ties to even, and held
    in float64 again.  A library that stores values as bfloat16 sees exactly
    this matrix, so an FP64 reference run on it isolates the error of the
    low-precision arithmetic from the change of the matrix.  Values must be
    finite and inside the float32 normal range (or zero)."""
    v = np.ascontiguousarray(a.values, dtype=np.float64)
    fin = np.abs(v[v != 0.0])
    if fin.size and (not np.all(np.isfinite(fin)) or fin.min() < 2.0 ** -126
                     or fin.max() >= 2.0 ** 127):
        raise ValueError("round_values_bf16: values outside the float32 normal range")
    bits = v.view(np.uint64)
    drop = np.uint64(45)                      # 52 - 7 mantissa bits dropped
    low = bits & np.uint64((1 << 45) - 1)
    half = np.uint64(1 << 44)
    keep = bits >> drop
    up = (low > half) | ((low == half) & ((keep & np.uint64(1)) == np.uint64(1)))
    keep = keep + up.astype(np.uint64)        # a carry moves into the exponent
    out = (keep << drop).view(np.float64)
    return Csr(n=a.n, row_ptr=a.row_ptr, col_idx=a.col_idx, values=out.copy(),
               name=a.name + "_bf16")


def csr_digest(a: Csr) -> str:
    """Content hash of a CSR matrix (checks that stored expected values were
    produced from the very same input)."""
    import hashlib
    h = hashlib.sha256()
    h.update(np.int64(a.n).tobytes())
    h.update(np.ascontiguousarray(a.row_ptr, dtype=np.int32).tobytes())
    h.update(np.ascontiguousarray(a.col_idx, dtype=np.int32).tobytes())
    h.update(np.ascontiguousarray(a.values, dtype=np.float64).tobytes())
    return h.hexdigest()[:16]


def request_stream(n_requests: int = 512, seed: int = 1, rate_hz: float = 1.0,
                   n_min: float = 1e4, n_max: float = 2e6):
    """Serving workload: request descriptors with Poisson arrival times.

    Each request: kind uniform over {lap2d, lap3d, wendland}; n log-uniform in
    [n_min, n_max] (2D: N = round(sqrt n), 3D: N = round(cbrt n)); shift or
    nugget log-uniform in [1e-3, 1]; Krylov steps uniform in 20..60;
    30 probes (sketch 10 + 20 residual); window 2.  Arrival gaps are
    exponential with mean 1/rate_hz (seconds).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    kinds = ("lap2d", "lap3d", "wendland")
    out = []
    t = 0.0
    for i in range(n_requests):
        kind = kinds[int(rng.integers(0, 3))]
        n = math.exp(rng.uniform(math.log(n_min), math.log(n_max)))
        shift = math.exp(rng.uniform(math.log(1e-3), 0.0))
        steps = int(rng.integers(20, 61))
        t += float(rng.exponential(1.0 / rate_hz))
        if kind == "lap2d":
            size = max(2, int(round(math.sqrt(n))))
        elif kind == "lap3d":
            size = max(2, int(round(n ** (1.0 / 3.0))))
        else:
            size = int(round(n))
        out.append(dict(id=i, kind=kind, size=size, shift=shift,
                        krylov_steps=steps, n_probes=30, sketch_rank=10,
                        iop_window=2, arrival_s=t))
    return out


def build_request_matrix(req) -> Csr:
    """Matrix for one request descriptor from request_stream()."""
    if req["kind"] == "lap2d":
        return lap2d(req["size"], req["shift"])
    if req["kind"] == "lap3d":
        return lap3d(req["size"], req["shift"])
    return wendland(req["size"], 48.0, req["shift"], seed=req["id"] + 1000)
