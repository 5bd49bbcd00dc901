"""Pins of the oracle's 7x7 median filter and start-point rules."""

import numpy as np
import pytest
from scipy import ndimage

import oracle


@pytest.mark.parametrize("shape", [(1, 1), (3, 5), (7, 7), (9, 100), (40, 13), (2500, 220)])
def test_median7x7_matches_scipy(shape):
    rng = np.random.default_rng(shape[0] * 1000 + shape[1])
    y = rng.random(shape).astype(np.float32)
    got = oracle.median7x7(y, chunk=1000)
    want = ndimage.median_filter(y, size=7, mode="nearest")
    assert np.array_equal(got, want)


def test_median7x7_with_ties_matches_scipy():
    rng = np.random.default_rng(11)
    y = rng.integers(0, 4, size=(50, 30)).astype(np.float32)
    assert np.array_equal(oracle.median7x7(y), ndimage.median_filter(y, size=7, mode="nearest"))


def test_start_point_on_rectangular_dip():
    """A flat image with a rectangular dip of width >= 4 survives the 7x7 median
    unchanged, so the start point is known in closed form."""
    f, k = 20, 60
    base, low, a, w = 1.25, 0.5, 21, 10
    y = np.full((f, k), base, dtype=np.float32)
    y[:, a:a + w] = low
    p0 = oracle.initial_guess(y)
    assert np.all(p0[:, 0] == a)                      # first (lowest) index of the minimum
    assert np.all(p0[:, 3] == np.float32(base))
    d = np.float32(1) - np.float32(np.float32(low) / np.float32(base))
    assert np.all(p0[:, 2] == d)
    assert np.all(p0[:, 1] == w)


def test_start_point_clips_and_floors():
    f, k = 8, 30
    y = np.full((f, k), 2.0, dtype=np.float32)
    y[:, 10:15] = 0.0                                  # depth 1 -> clipped to 0.95
    p0 = oracle.initial_guess(y)
    assert np.all(p0[:, 2] == np.float32(0.95))
    y = np.full((f, k), 2.0, dtype=np.float32)        # no dip -> depth 0 -> 0.05, width floor 2
    p0 = oracle.initial_guess(y)
    assert np.all(p0[:, 2] == np.float32(0.05))
    assert np.all(p0[:, 1] == 2)
    assert np.all(p0[:, 0] == 0)
    z = np.zeros((f, k), dtype=np.float32)             # b0 = 0 -> depth 0.05
    p0 = oracle.initial_guess(z)
    assert np.all(p0[:, 2] == np.float32(0.05)) and np.all(p0[:, 3] == 0)


def test_lower_median_even_count():
    """b0 is the lower median: for K even the smaller of the two middle values."""
    k = 10
    row = np.arange(k, dtype=np.float32)[::-1] + 1.0   # 10..1
    y = np.tile(row, (9, 1))
    m = oracle.median7x7(y)
    p0 = oracle.initial_guess(y)
    assert np.all(p0[:, 3] == np.sort(m[0])[(k - 1) // 2])


def test_width_count_is_strictly_below_half_depth():
    """Teeth whose filtered value equals the half-depth level b0 (1 - d0/2)
    exactly are not counted in the start width."""
    f, k = 12, 60
    y = np.full((f, k), 1.0, dtype=np.float32)
    y[:, 20:28] = 0.5          # dip: d0 = 0.5, half-depth level 0.75 exactly
    y[:, 40:46] = 0.75         # plateau exactly at the level
    p0 = oracle.initial_guess(y)
    assert np.all(p0[:, 2] == np.float32(0.5))
    assert np.all(p0[:, 1] == 8)
