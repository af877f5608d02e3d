"""Pins of the oracle's Philox4x64-10 and Rademacher layout (CPU only)."""
import os

import numpy as np
import pytest

from oracle import philox4x64_10, philox4x64_10_np, rademacher

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x64_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        w = [int(x, 16) for x in line.split()]
        rows.append((tuple(w[0:4]), tuple(w[4:6]), tuple(w[6:10])))
    return rows


def test_known_answer_vectors():
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, out in rows:
        assert philox4x64_10(ctr, key) == out


def test_matches_numpy_philox():
    # numpy's Philox advances the counter before producing a block, so the
    # block at counter c is the first output of a generator started at c - 1.
    rng = np.random.Generator(np.random.PCG64(123))
    for _ in range(20):
        c = int(rng.integers(1, 2**62)) | (int(rng.integers(0, 2**62)) << 64)
        key = [int(rng.integers(0, 2**63)), int(rng.integers(0, 2**63))]
        words = [(c >> (64 * i)) & ((1 << 64) - 1) for i in range(4)]
        ref = np.random.Philox(counter=c - 1, key=key).random_raw(4)
        assert philox4x64_10(words, key) == tuple(int(x) for x in ref)


def test_vectorised_equals_scalar():
    rng = np.random.Generator(np.random.PCG64(7))
    c = rng.integers(0, 2**63, size=(4, 16), dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    k0, k1 = 0xDEADBEEFCAFEF00D, 0x0123456789ABCDEF
    out = philox4x64_10_np(c[0], c[1], c[2], c[3], k0, k1)
    for i in range(16):
        ref = philox4x64_10([int(c[j, i]) for j in range(4)], (k0, k1))
        assert tuple(int(o[i]) for o in out) == ref


def test_rademacher_bit_layout():
    seed, n = 42, 1000
    s = rademacher(seed, n, 3, 6)
    assert s.shape == (n, 3)
    assert set(np.unique(s)) <= {-1.0, 1.0}
    for p in (3, 4, 5):
        for i in (0, 1, 63, 64, 200, 255, 256, 511, 777, 999):
            words = philox4x64_10((i // 256, p, 0, 0), (seed, 0))
            bit = (words[(i // 64) % 4] >> (i % 64)) & 1
            assert s[i, p - 3] == (-1.0 if bit else 1.0)


def test_rademacher_columns_are_independent_of_range():
    a = rademacher(9, 777, 0, 8)
    b = rademacher(9, 777, 5, 8)
    np.testing.assert_array_equal(a[:, 5:], b)
    # a different seed gives a different matrix; +-1 balanced
    c = rademacher(10, 777, 0, 8)
    assert np.mean(a != c) > 0.4
    big = rademacher(3, 20000, 0, 4)
    assert abs(big.mean()) < 0.02


# ---------------------------------------------------------------------------
# Gaussian probes: Box-Muller on the Philox stream with counter word 2 = 1.
# ---------------------------------------------------------------------------
from oracle.philox import gaussian, probes, PROBE_GAUSSIAN, PROBE_RADEMACHER  # noqa: E402


def _numpy_block(seed, b, p, c2):
    # independent Philox implementation: numpy's generator at counter c - 1
    c = b | (p << 64) | (c2 << 128)
    return [int(x) for x in np.random.Philox(counter=c - 1, key=[seed, 0]).random_raw(4)]


def test_gaussian_pairs_follow_numpy_philox_words():
    # every pair of rows (4b + 2j, 4b + 2j + 1) carries radius^2 = -2 log u1 and
    # angle 2 pi u2 of words (2j, 2j + 1) of the block at counter (b, p, 1, 0):
    # a wrong counter word, word pairing or sin/cos assignment fails here
    seed = 0x1234_5678_9ABC
    g = gaussian(seed, 4 * 7 + 2, 3, 6)  # ragged tail: 30 rows
    for col in range(3):
        p = 3 + col
        for b in range(8):
            w = _numpy_block(seed, b, p, 1)
            for pair in range(2):
                r0 = 4 * b + 2 * pair
                if r0 + 1 >= g.shape[0]:
                    continue
                u1 = ((w[2 * pair] >> 11) + 1) * 2.0**-53
                u2 = (w[2 * pair + 1] >> 11) * 2.0**-53
                ze, zo = g[r0, col], g[r0 + 1, col]
                assert ze * ze + zo * zo == pytest.approx(-2.0 * np.log(u1), rel=1e-13)
                ang = np.arctan2(zo, ze) % (2 * np.pi)
                assert ang == pytest.approx(2 * np.pi * u2, abs=1e-12) or \
                    abs(ang - 2 * np.pi * u2) > 2 * np.pi - 1e-12


def test_gaussian_distribution():
    # N(0, 1): Kolmogorov-Smirnov, moments, no correlation between columns
    import scipy.stats as st
    g = gaussian(11, 400_000, 0, 3)
    for j in range(3):
        assert st.kstest(g[:, j], "norm").pvalue > 1e-3
    assert np.all(np.abs(g.mean(axis=0)) < 0.01)
    assert np.all(np.abs(g.var(axis=0) - 1.0) < 0.01)
    assert np.all(np.abs(st.kurtosis(g, axis=0, fisher=False) - 3.0) < 0.05)
    c = np.corrcoef(g.T)
    assert np.all(np.abs(c - np.eye(3)) < 0.01)


def test_gaussian_columns_are_independent_of_range():
    a = gaussian(5, 1001, 0, 6)
    b = gaussian(5, 1001, 2, 5)
    np.testing.assert_array_equal(a[:, 2:5], b)
    np.testing.assert_array_equal(probes(5, 1001, 2, 5, PROBE_GAUSSIAN), b)
    np.testing.assert_array_equal(probes(5, 1001, 2, 5, PROBE_RADEMACHER), rademacher(5, 1001, 2, 5))
