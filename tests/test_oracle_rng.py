"""Pins of the counter-based sketch generator (CPU).

The H^2 construction draws its Gaussian sketch from SplitMix64 and the
Box-Muller transform on both sides, so the generator is pinned to the
published definitions rather than to itself:

* SplitMix64 started from state 0 produces the sequence listed with Vigna's
  reference implementation (xoshiro/splitmix64.c test outputs), whose first
  four values are below;
* the normals have the moments and distribution of N(0, 1), and entry (t, j)
  of the sketch depends only on its counter (t << 24) | j.
"""
import numpy as np
import pytest
from scipy import stats

from oracle import rng

# SplitMix64, seed 0: the first four outputs (state advanced before mixing)
SPLITMIX64_SEED0 = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]


def test_splitmix64_published_sequence():
    states = np.arange(4, dtype=np.uint64)
    with np.errstate(over="ignore"):
        states = states * np.uint64(0x9E3779B97F4A7C15)
    out = [int(v) for v in rng.splitmix64(states)]
    assert out == SPLITMIX64_SEED0


def test_normal_moments_and_distribution():
    z = rng.normal(0x5EEDF00D, np.arange(1 << 20, dtype=np.uint64))
    assert np.all(np.isfinite(z))
    n = z.size
    # mean, variance, skewness and excess kurtosis of N(0, 1), each within
    # five standard errors of a sample of 2^20
    assert abs(z.mean()) < 5 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0 / n)
    assert abs(stats.skew(z)) < 5 * np.sqrt(6.0 / n)
    assert abs(stats.kurtosis(z)) < 5 * np.sqrt(24.0 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # tails: P(|z| > 3) = 2.70e-3
    frac = np.mean(np.abs(z) > 3.0)
    assert abs(frac - 2.6998e-3) < 5 * np.sqrt(2.6998e-3 / n)


def test_seeds_and_counters_decorrelate():
    c = np.arange(1 << 16, dtype=np.uint64)
    a = rng.normal(1, c)
    b = rng.normal(2, c)
    assert abs(np.corrcoef(a, b)[0, 1]) < 5 / np.sqrt(c.size)
    assert abs(np.corrcoef(a[:-1], a[1:])[0, 1]) < 5 / np.sqrt(c.size)


@pytest.mark.parametrize("rows,cols", [(3, 5), (40, 7)])
def test_sketch_entries_follow_their_counters(rows, cols):
    seed = 12345
    S = rng.sketch(rows, cols, seed)
    t = np.arange(rows, dtype=np.uint64)[:, None]
    j = np.arange(cols, dtype=np.uint64)[None, :]
    assert np.array_equal(S, rng.normal(seed, (t << np.uint64(24)) | j))
    # a larger request leaves the leading block unchanged
    big = rng.sketch(rows + 9, cols + 3, seed)
    assert np.array_equal(big[:rows, :cols], S)
    assert not S.flags.writeable
