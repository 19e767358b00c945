"""SplitMix64: published output sequence for state 0 (Steele, Lea & Flood 2014;
the reference C generator seeded with 0 returns 0xE220A8397B1DCDAF,
0x6E789E6AA1B965F4, ...)."""
import numpy as np

from oracle import rng


def test_splitmix64_published_sequence():
    g = 0x9E3779B97F4A7C15
    out = rng.splitmix64(np.array([0, g], dtype=np.uint64))
    assert int(out[0]) == 0xE220A8397B1DCDAF
    assert int(out[1]) == 0x6E789E6AA1B965F4


def test_uniform_range_and_moments():
    v = rng.uniform_pm1(7, np.arange(200000))
    assert v.min() >= -1 and v.max() < 1
    assert abs(v.mean()) < 0.01 and abs((v ** 2).mean() - 1 / 3) < 0.01
    assert not np.array_equal(v, rng.uniform_pm1(8, np.arange(200000)))
