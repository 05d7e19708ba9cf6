"""Pins of the seeded input generator (shared by the oracle and the GPU runs)."""
import numpy as np
import pytest
from scipy import stats


def test_philox_known_answers(datagen_mod):
    # Known-answer vectors published with Random123 (Salmon et al., SC'11) for
    # Philox4x32 with 10 rounds: (counter, key) -> output.
    kat = [
        ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
        ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
        ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
         (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
    ]
    for ctr, key, want in kat:
        assert tuple(int(v) for v in datagen_mod.philox4x32_10(ctr, key)) == want


def test_gaussians_are_standard_normal(datagen_mod):
    g = np.concatenate([datagen_mod.gaussians(7, 0, r, 4096) for r in range(64)])
    assert abs(g.mean()) < 0.01 and abs(g.std() - 1.0) < 0.01
    assert stats.kstest(g, "norm").pvalue > 1e-3
    # skewness ~ 0, kurtosis ~ 3
    assert abs(stats.skew(g)) < 0.03 and abs(stats.kurtosis(g, fisher=False) - 3.0) < 0.06


def test_random_walk_recurrence(datagen_mod):
    # Experimental Evaluation, Datasets: first point an N(0,1) draw, then each
    # point adds a fresh N(0,1) draw to the previous one.
    n, length = 8, 256
    x = datagen_mod.random_walks(n, length, seed=11, stream=0)
    for r in range(n):
        g = datagen_mod.gaussians(11, 0, r, length)
        want = np.cumsum(g)  # fp64 running sum, same left-to-right order
        np.testing.assert_array_equal(x[r], want.astype(np.float32))


def test_rows_are_addressable(datagen_mod):
    a = datagen_mod.random_walks(100, 64, seed=5, stream=0)
    b = datagen_mod.random_walks(10, 64, seed=5, stream=0, row0=37)
    np.testing.assert_array_equal(a[37:47], b)
    c = datagen_mod.random_walks(100, 64, seed=5, stream=0, nthreads=3)
    np.testing.assert_array_equal(a, c)


def test_mixture_shape_and_range(datagen_mod):
    cen = datagen_mod.mixture_centres(50, 32)
    assert cen.min() >= 0.0 and cen.max() <= 255.0
    m = datagen_mod.mixture(500, 32, cen)
    assert m.min() >= 0 and m.max() <= 255
    np.testing.assert_array_equal(m, np.round(m))


def test_noise_queries(datagen_mod):
    base = np.zeros((4, 16), dtype=np.float32)
    q = datagen_mod.add_noise(base, [0.0, 0.01, 0.1, 1.0])
    assert np.all(q[0] == 0)
    for i, s in enumerate([0.01, 0.1, 1.0], start=1):
        g = datagen_mod.gaussians(datagen_mod.SEED_NOISE, datagen_mod.STREAM_NOISE, i, 16)
        np.testing.assert_array_equal(q[i], (s * g).astype(np.float32))


def test_uniform_ints_in_range(datagen_mod):
    v = datagen_mod.uniform_ints(10000, 1000, 3, 9)
    assert v.min() >= 0 and v.max() < 1000
    assert len(np.unique(v)) > 990
