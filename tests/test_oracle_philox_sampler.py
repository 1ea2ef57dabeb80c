"""Pins for the oracle's random inputs: Philox4x64-10, Gaussian G_n, RANDSAMPLE.

What fixes each function other than itself:
* philox4x64: the published known-answer vector (tests/golden) and numpy's
  independent Philox 4x64 bit generator on random counters and keys;
* gaussian_matrix: distribution tests (Kolmogorov-Smirnov against N(0,1),
  moments, pair independence) and the column-major counter layout;
* sampling_weights / draw_columns: exact big-integer definitions of the draw,
  a brute-force search for xi, the closed form 1/sqrt(T p~) of the rescale,
  and a chi-squared test of the empirical draw frequencies against w / W.
"""
import math
import os

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle.philox import MASK64, philox4x64

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_published_kat():
    with open(os.path.join(GOLDEN, "philox4x64_10_kat.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    assert rows
    for r in rows:
        v = [int(x, 16) for x in r]
        assert philox4x64(v[0:4], v[4:6]) == tuple(v[6:10])


def _numpy_block(counter, key):
    # numpy's Philox increments its 256-bit counter before producing a block.
    c = sum(int(w) << (64 * i) for i, w in enumerate(counter))
    k = int(key[0]) | (int(key[1]) << 64)
    g = np.random.Philox(counter=(c - 1) % (1 << 256), key=k)
    return tuple(int(x) for x in g.random_raw(4))


def test_philox_matches_numpy_random_counters_and_keys():
    rng = np.random.default_rng(123)
    for trial in range(200):
        ctr = [int(x) for x in rng.integers(0, 2**63, size=4, dtype=np.int64)]
        ctr = [(c << 1 | (trial & 1)) & MASK64 for c in ctr]
        key = [int(x) for x in rng.integers(0, 2**63, size=2, dtype=np.int64)]
        if trial % 7 == 0:
            ctr[0] = 0  # exercise the borrow across words in the numpy side
        assert philox4x64(ctr, key) == _numpy_block(ctr, key)


def test_philox_structured_counters_used_by_the_method():
    for b in (0, 1, 2, 1000, 2**40 + 3):
        for mode in (0, 1, 7):
            for tag in (oracle.TAG_GAUSS, oracle.TAG_SAMPLE):
                for seed in (0, 1, 2**64 - 1):
                    ctr = (b, mode, tag, 0)
                    assert philox4x64(ctr, (seed, 0)) == _numpy_block(ctr, (seed, 0))


def test_gaussian_layout_is_column_major_stream():
    a = oracle.gaussian_matrix(10, 3, 0, 5).ravel(order="F")
    b = oracle.gaussian_matrix(30, 1, 0, 5).ravel(order="F")
    c = oracle.gaussian_matrix(6, 5, 0, 5).ravel(order="F")
    assert np.array_equal(a, b)
    assert np.array_equal(a, c[:30])
    assert not np.array_equal(a, oracle.gaussian_matrix(10, 3, 1, 5).ravel("F"))
    assert not np.array_equal(a, oracle.gaussian_matrix(10, 3, 0, 6).ravel("F"))


def test_gaussian_box_muller_against_philox_words():
    # First element of block 0 from the raw Philox words, via the polar form of
    # Box-Muller (rho, theta), checked against an independent route:
    # z_a^2 + z_b^2 = -2 ln u1 and atan2(z_b, z_a) = 2 pi u2 (mod 2 pi).
    G = oracle.gaussian_matrix(4, 1, 3, 11).ravel(order="F")
    r = philox4x64((0, 3, oracle.TAG_GAUSS, 0), (11, 0))
    for pair in range(2):
        ra, rb = r[2 * pair], r[2 * pair + 1]
        u1 = ((ra >> 11) + 1) / 2.0**53
        u2 = (rb >> 11) / 2.0**53
        za, zb = G[2 * pair], G[2 * pair + 1]
        assert math.isclose(za * za + zb * zb, -2.0 * math.log(u1), rel_tol=1e-13)
        ang = math.atan2(zb, za) % (2 * math.pi)
        assert math.isclose(ang, (2 * math.pi * u2) % (2 * math.pi), abs_tol=1e-12)


def test_gaussian_distribution():
    G = oracle.gaussian_matrix(400, 50, 2, 99).ravel(order="F")
    assert abs(G.mean()) < 5 / math.sqrt(G.size)
    assert abs(G.var() - 1.0) < 5 * math.sqrt(2.0 / G.size)
    assert stats.kstest(G, "norm").pvalue > 1e-3
    # the two halves of each Box-Muller pair are uncorrelated
    a, b = G[0::2], G[1::2]
    assert abs(np.corrcoef(a, b)[0, 1]) < 5 / math.sqrt(a.size)


def test_ceil_log2():
    for J in range(1, 5000):
        assert oracle.ceil_log2(J) == math.ceil(math.log2(J))
    assert oracle.ceil_log2(2**40) == 40 and oracle.ceil_log2(2**40 + 1) == 41


def test_weights_rules():
    J = 1000
    rng = np.random.default_rng(0)
    n = rng.random(J) ** 4
    n[5] = 0.0
    n[6] = 1e-300          # non-zero but tiny: weight floor of 1
    w = oracle.sampling_weights(n, J, oracle.PROB_NEARLY_OPTIMAL)
    k = 60 - oracle.ceil_log2(J)
    assert w.dtype == np.uint64
    assert int(w[np.argmax(n)]) == 2**k
    assert int(w[5]) == 0 and int(w[6]) == 1
    assert int(w.astype(object).sum()) <= 2**60
    # p~ = w / W is within the quantisation step of n / sum(n)
    W = float(w.astype(object).sum())
    p = n / n.sum()
    pt = w.astype(np.float64) / W
    big = n > 1e-6 * n.max()
    assert np.all(np.abs(pt[big] / p[big] - 1) < 1e-9)
    assert np.array_equal(oracle.sampling_weights(None, 7, oracle.PROB_UNIFORM),
                          np.ones(7, dtype=np.uint64))
    with pytest.raises(FloatingPointError):
        oracle.sampling_weights(np.zeros(4), 4, oracle.PROB_NEARLY_OPTIMAL)
    with pytest.raises(FloatingPointError):
        oracle.sampling_weights(np.array([1.0, np.nan]), 2, oracle.PROB_NEARLY_OPTIMAL)


def test_draw_definition_exact():
    rng = np.random.default_rng(1)
    J, T, seed, mode = 37, 301, 77, 2
    w = rng.integers(0, 2**20, size=J).astype(np.uint64)
    w[3] = 0
    xi, scale, W = oracle.draw_columns(w, T, seed, mode)
    cdf = [0]
    for v in w:
        cdf.append(cdf[-1] + int(v))
    assert W == cdf[-1]
    for t in range(T):
        r = philox4x64((t // 2, mode, oracle.TAG_SAMPLE, 0), (seed, 0))
        h, l = r[2 * (t % 2)], r[2 * (t % 2) + 1]
        x = (((h << 64) | l) * W) >> 128          # floor(U * W), U = 128-bit fraction
        assert 0 <= x < W
        # brute-force search: first column whose inclusive prefix exceeds x
        j = next(j for j in range(J) if cdf[j + 1] > x)
        assert xi[t] == j
        assert int(w[j]) > 0
        exact = 1.0 / math.sqrt(T * int(w[j]) / W)
        assert math.isclose(scale[t], exact, rel_tol=4e-16)
        assert scale[t] == math.sqrt((float(W) / float(int(w[j]))) / float(T))


def test_uniform_draw_is_the_scaled_integer():
    J, T = 1000, 500
    xi, scale, W = oracle.draw_columns(np.ones(J, dtype=np.uint64), T, 4, 0)
    assert W == J
    for t in range(T):
        r = philox4x64((t // 2, 0, oracle.TAG_SAMPLE, 0), (4, 0))
        h, l = r[2 * (t % 2)], r[2 * (t % 2) + 1]
        assert xi[t] == (((h << 64) | l) * J) >> 128
    assert np.all(scale == math.sqrt(J / T))


def test_draw_frequencies_chi_squared():
    J = 12
    w = np.array([1, 2, 3, 4, 0, 6, 7, 8, 9, 10, 30, 100], dtype=np.uint64) * 1000
    T = 60000
    xi, _, W = oracle.draw_columns(w, T, 2024, 1)
    counts = np.bincount(xi, minlength=J)
    assert counts[4] == 0
    keep = w > 0
    expected = T * w[keep].astype(np.float64) / W
    chi2 = stats.chisquare(counts[keep], expected)
    assert chi2.pvalue > 1e-3


def test_randsample_modes_and_seeds_differ():
    a = oracle.randsample(None, 10**6, 64, oracle.PROB_UNIFORM, 1, 0)[0]
    b = oracle.randsample(None, 10**6, 64, oracle.PROB_UNIFORM, 1, 1)[0]
    c = oracle.randsample(None, 10**6, 64, oracle.PROB_UNIFORM, 2, 0)[0]
    assert not np.array_equal(a, b) and not np.array_equal(a, c)
