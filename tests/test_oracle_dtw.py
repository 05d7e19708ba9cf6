"""Pins of the oracle's DTW search (the paper's closing experiment: the same
index searched with the LB_Keogh envelope of the query, warping window 10%
of the length).

  * a hand-worked example (a shifted ramp) and its Euclidean counterpart;
  * r = 0 is the canonical squared Euclidean distance bit for bit;
  * on tiny inputs, the minimum over every warping path in the band (listed
    one by one) equals the recurrence exactly;
  * DTW <= ED, non-increasing in r, symmetric, and the full band equals the
    unconstrained textbook DP;
  * LB_Keogh <= DTW, equal to ED at r = 0; the index bound <= LB_Keogh;
  * the index search equals brute force (the pruning is safe).
"""
import itertools

import numpy as np
import pytest


def test_dtw_hand_example(oracle_mod):
    # x is q shifted right by one: the path (0,0) (0,1) (1,2) (2,3) (3,4) (4,4)
    # costs 0 + 0 + 0 + 0 + 0 + (4 - 3)^2 = 1; the diagonal costs 4 x 1
    q = np.array([0, 1, 2, 3, 4], np.float32)
    x = np.array([0, 0, 1, 2, 3], np.float32)
    assert oracle_mod.dtw64(q, x, 1) == 1.0
    assert oracle_mod.dtw64(q, x, 0) == 4.0
    assert oracle_mod.dtw64(q, x, 4) == 1.0
    # a spike matched against a flat series: every path meets the spike once
    s = np.array([0, 0, 5, 0, 0], np.float32)
    z = np.zeros(5, np.float32)
    assert oracle_mod.dtw64(s, z, 2) == 25.0


def test_dtw_band_zero_is_the_canonical_ed(oracle_mod, datagen_mod):
    x = oracle_mod.znorm(datagen_mod.random_walks(40, 100, seed=8))
    for i in range(0, 40, 2):
        assert oracle_mod.dtw64(x[i], x[i + 1], 0) == oracle_mod.d64(x[i], x[i + 1])


def _paths(n, r):
    """Every monotone path from (0,0) to (n-1,n-1) with |i - j| <= r."""
    out = []

    def walk(i, j, acc):
        if (i, j) == (n - 1, n - 1):
            out.append(acc)
            return
        for di, dj in ((1, 0), (0, 1), (1, 1)):
            a, b = i + di, j + dj
            if a < n and b < n and abs(a - b) <= r:
                walk(a, b, acc + [(a, b)])

    walk(0, 0, [(0, 0)])
    return out


@pytest.mark.parametrize("n,r", [(4, 1), (5, 1), (5, 2), (6, 5), (6, 2)])
def test_dtw_equals_the_best_path(oracle_mod, n, r):
    rng = np.random.default_rng(n * 10 + r)
    paths = _paths(n, r)
    for _ in range(20):
        # small integers: every path sum is exact in fp64, so the minimum is too
        q = rng.integers(-4, 5, n).astype(np.float32)
        x = rng.integers(-4, 5, n).astype(np.float32)
        best = min(sum((float(q[i]) - float(x[j])) ** 2 for i, j in p) for p in paths)
        assert oracle_mod.dtw64(q, x, r) == best


def test_dtw_properties(oracle_mod, datagen_mod):
    z = oracle_mod.znorm(datagen_mod.random_walks(60, 64, seed=9))
    for i in range(0, 60, 2):
        q, x = z[i], z[i + 1]
        vals = [oracle_mod.dtw64(q, x, r) for r in (0, 1, 3, 6, 12, 63)]
        assert all(a >= b for a, b in zip(vals, vals[1:]))  # wider band, smaller or equal
        assert vals[0] == oracle_mod.d64(q, x)
        assert oracle_mod.dtw64(x, q, 6) == oracle_mod.dtw64(q, x, 6)
        assert oracle_mod.dtw64(q, x, 1000) == vals[-1]  # beyond L - 1: unconstrained


def test_dtw_full_band_is_the_unconstrained_dp(oracle_mod):
    """The unconstrained textbook DP over the whole matrix (numpy, fp64)."""
    rng = np.random.default_rng(3)
    for n in (1, 2, 7, 16):
        q = rng.standard_normal(n).astype(np.float32)
        x = rng.standard_normal(n).astype(np.float32)
        D = np.full((n + 1, n + 1), np.inf)
        D[0, 0] = 0.0
        for i in range(1, n + 1):
            for j in range(1, n + 1):
                d = np.float64(q[i - 1]) - np.float64(x[j - 1])
                D[i, j] = d * d + min(D[i - 1, j], D[i, j - 1], D[i - 1, j - 1])
        assert oracle_mod.dtw64(q, x, n - 1) == D[n, n]


def test_envelope_and_lb_keogh(oracle_mod, datagen_mod):
    q = np.array([0, 3, 1, -2, 5, 4], np.float32)
    up, lo = oracle_mod.envelope(q, 1)
    np.testing.assert_array_equal(up, [3, 3, 3, 5, 5, 5])
    np.testing.assert_array_equal(lo, [0, 0, -2, -2, -2, 4])
    z = oracle_mod.znorm(datagen_mod.random_walks(200, 128, seed=10))
    for i in range(0, 200, 2):
        q, x = z[i], z[i + 1]
        assert oracle_mod.lb_keogh(q, x, 0) == oracle_mod.d64(q, x)
        for r in (1, 12, 40):
            lbk = oracle_mod.lb_keogh(q, x, r)
            assert lbk <= oracle_mod.dtw64(q, x, r) * (1 + 1e-12)
            assert lbk <= oracle_mod.lb_keogh(q, x, r - 1) * (1 + 1e-12)  # wider envelope, looser bound


def test_index_bound_below_lb_keogh(oracle_mod, datagen_mod):
    """The DTW bound of a series' own full-cardinality word never exceeds its
    LB_Keogh (with the word's regions widened by the PAA rounding slack), and
    coarser nodes give smaller bounds."""
    L, w, b = 128, 16, 8
    z = oracle_mod.znorm(datagen_mod.random_walks(300, L, seed=11))
    words = oracle_mod.words(z, w, b)
    slack = 6 * 2.0 ** -23 * float(np.abs(z).max())
    full = np.full(w, b, np.uint8)
    half = np.full(w, 4, np.uint8)
    for i in range(0, 300, 3):
        q, x = z[i], z[i + 1]
        for r in (0, 3, 12):
            lbk = oracle_mod.lb_keogh(q, x, r)
            md = oracle_mod.mindist_dtw_sq(q, r, full, words[i + 1], b, w, slack)
            assert md <= lbk * (1 + 1e-12)
            coarse = oracle_mod.mindist_dtw_sq(q, r, half, words[i + 1] >> 4, b, w, slack)
            assert coarse <= md * (1 + 1e-12)


@pytest.mark.parametrize("k,band", [(1, 6), (5, 6), (3, 0), (2, 31)])
def test_isax_dtw_search_equals_brute_force(oracle_mod, datagen_mod, k, band):
    n, L, w, b, cap = 3000, 64, 16, 8, 50
    z = oracle_mod.znorm(datagen_mod.random_walks(n, L, seed=12))
    words = oracle_mod.words(z, w, b)
    leaves, pos = oracle_mod.build_leaves(words, b, cap)
    fresh = oracle_mod.znorm(datagen_mod.random_walks(4, L, seed=13))
    noisy = datagen_mod.add_noise(z[[5, 2000]], [0.1, 1.0])
    q = np.concatenate([fresh, noisy]).astype(np.float32)
    bi, bd, _ = oracle_mod.knn_brute_dtw(z, q, k, band, nthreads=8)
    ii, idd, _, st = oracle_mod.knn_isax_dtw(z, words, b, leaves, pos, q, k, band, return_stats=True)
    np.testing.assert_array_equal(ii, bi)
    np.testing.assert_array_equal(idd, bd)
    if band <= 6:  # the bounds prune (a sigma = 1 query, or a wide band, may visit everything)
        assert st[:, 3].sum() < n * len(q) / 2
