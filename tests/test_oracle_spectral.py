"""Pins of the spectral interval and the shift rules (CPU only)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import (GERSH_FLOOR_REL, gershgorin_bounds, osa_iop_shift, oslq_scaling,
                    spectral_interval)


def test_gershgorin_closed_form_laplacians():
    # interior rows of the 2D (3D) Dirichlet Laplacian give 4+s +- 4 (6+s +- 6)
    lo, hi = gershgorin_bounds(W.lap2d(9, 0.1))
    assert lo == pytest.approx(0.1, abs=1e-14) and hi == pytest.approx(8.1, abs=1e-14)
    lo, hi = gershgorin_bounds(W.lap3d(5, 1e-3))
    assert lo == pytest.approx(1e-3, abs=1e-14) and hi == pytest.approx(12.001, abs=1e-14)


def test_gershgorin_brute_force_dense():
    q = W.random_spd_dense(9, seed=3)
    a = W.from_dense(q)
    lo, hi = gershgorin_bounds(a)
    rad = np.sum(np.abs(q), axis=1) - np.abs(np.diag(q))
    assert lo == pytest.approx(float(np.min(np.diag(q) - rad)), rel=1e-13)
    assert hi == pytest.approx(float(np.max(np.diag(q) + rad)), rel=1e-13)
    # the interval encloses the spectrum
    lam = np.linalg.eigvalsh(q)
    assert lo <= lam.min() and lam.max() <= hi


def test_er_laplacian_lower_bound_is_shift():
    a = W.er_laplacian(2000, 16000, seed=0, shift=0.05)
    assert a.nnz == 2000 + 2 * 16000
    lo, hi = gershgorin_bounds(a)
    assert lo == pytest.approx(0.05, abs=1e-12)


def test_floor_and_hints():
    # a Wendland kernel matrix is not diagonally dominant: Gershgorin lower
    # bound is negative and the floor takes over unless a hint is given
    a = W.wendland(400, 20.0, 1e-2, seed=1)
    glo, ghi = gershgorin_bounds(a)
    assert glo < 0
    lo, hi = spectral_interval(a)
    assert hi == ghi and lo == pytest.approx(GERSH_FLOOR_REL * ghi)
    lo, hi = spectral_interval(a, lo_hint=1e-2)
    assert lo == 1e-2 and hi == ghi
    lo, hi = spectral_interval(a, lo_hint=1e-2, hi_hint=50.0)
    assert (lo, hi) == (1e-2, 50.0)


def test_shift_rules():
    # OSLQ: J = Q / lmax when lmin < 1, else J = Q
    assert oslq_scaling(0.1, 8.0) == (8.0, math.log(8.0))
    assert oslq_scaling(1.5, 8.0) == (1.0, 0.0)
    # OSA-IOP: gamma = sqrt(lo hi); c = log lo if lo < 1 else log gamma
    g, c = osa_iop_shift(0.25, 4.0)
    assert g == pytest.approx(1.0) and c == pytest.approx(math.log(0.25))
    g, c = osa_iop_shift(2.0, 8.0)
    assert g == pytest.approx(4.0) and c == pytest.approx(math.log(4.0))


def test_gamma_is_minimax_centre():
    # Proposition 2.1: gamma* = sqrt(lmin lmax) minimises max |log(lambda/gamma)|
    lo, hi = 0.03, 7.0
    g, _ = osa_iop_shift(lo, hi)
    grid = np.exp(np.linspace(math.log(lo), math.log(hi), 2001))
    worst = np.maximum(np.abs(np.log(lo / grid)), np.abs(np.log(hi / grid)))
    assert grid[np.argmin(worst)] == pytest.approx(g, rel=5e-3)
