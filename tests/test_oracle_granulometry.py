"""Pins of the oracle's granulometry, pattern spectrum and alternating
sequential filter (Eq. 16-20) against things other than the oracle:

- scipy.ndimage.grey_opening / grey_closing with a (2s+1)^2 flat square and
  nearest borders (edge replication equals the clipped window for each of
  the erosion and the dilation), for gamma_s, phi_s and the whole ASF;
- closed forms: squares of side a away from the border survive an opening
  of size s exactly when a >= 2s + 1, so G_s is a sum of square areas and
  the pattern spectrum puts each square's area at s = (a - 1) / 2; ASF_1
  removes isolated specks of either sign from a flat image;
- G is non-increasing in s and an opening is idempotent.
"""
from fractions import Fraction

import numpy as np
import pytest
from scipy import ndimage

import oracle

DTYPES = [np.uint8, np.float32, np.float64]


def rand_img(shape, dtype, seed, levels=8):
    v = np.random.default_rng(seed).integers(0, levels, size=shape)
    return (v * 30).astype(dtype) if dtype == np.uint8 else (v * 0.25 - 0.9).astype(dtype)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("shape", [(1, 9), (8, 1), (13, 17), (26, 21)])
@pytest.mark.parametrize("s", [0, 1, 2, 5])
def test_opening_closing_match_scipy(dtype, shape, s):
    f = rand_img(shape, dtype, seed=s + shape[0])
    size = (2 * s + 1, 2 * s + 1)
    assert np.array_equal(oracle.opening(f, s), ndimage.grey_opening(f, size=size, mode="nearest"))
    assert np.array_equal(oracle.closing(f, s), ndimage.grey_closing(f, size=size, mode="nearest"))


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("s_max", [0, 1, 3])
def test_asf_matches_scipy(dtype, s_max):
    f = rand_img((24, 31), dtype, seed=7 + s_max)
    g = f.copy()
    for s in range(1, s_max + 1):
        size = (2 * s + 1, 2 * s + 1)
        g = ndimage.grey_closing(ndimage.grey_opening(g, size=size, mode="nearest"), size=size,
                                 mode="nearest")
    assert np.array_equal(oracle.asf(f, s_max), g)


@pytest.mark.parametrize("dtype", DTYPES)
def test_granulometry_of_squares(dtype):
    f = np.zeros((60, 70), dtype=dtype)
    sides = {(5, 5): 1, (5, 20): 3, (5, 40): 5, (25, 5): 7, (25, 30): 9, (40, 50): 13}
    for (y, x), a in sides.items():
        f[y:y + a, x:x + a] = 2
    G, PS = oracle.granulometry(f, 8)
    for s in range(9):
        assert G[s] == sum(2 * a * a for a in sides.values() if a >= 2 * s + 1), s
    expect_ps = np.zeros(8)
    for a in sides.values():
        if (a - 1) // 2 < 8:
            expect_ps[(a - 1) // 2] += 2 * a * a
    assert np.array_equal(PS, expect_ps)


@pytest.mark.parametrize("dtype", DTYPES)
def test_asf_removes_specks(dtype):
    f = np.full((30, 40), 100, dtype=dtype)
    f[5, 7] = 200
    f[20, 33] = 0
    f[12, 20] = 150
    f[13, 21] = 50
    assert np.array_equal(oracle.asf(f, 1), np.full_like(f, 100))


@pytest.mark.parametrize("dtype", DTYPES)
def test_granulometry_invariants(dtype):
    f = rand_img((33, 29), dtype, seed=3)
    G, PS = oracle.granulometry(f, 6)
    # G_0 is the sum of f, rounded once: compare with exact rational arithmetic
    assert G[0] == float(sum(Fraction(float(x)) for x in f.ravel()))
    assert np.all(PS >= 0)
    for s in (1, 3):
        o = oracle.opening(f, s)
        assert np.all(o <= f)
        assert np.array_equal(oracle.opening(o, s), o)


def test_zero_sizes_and_empty():
    f = rand_img((9, 11), np.float32, seed=1)
    G, PS = oracle.granulometry(f, 0)
    assert G.shape == (1,) and PS.shape == (0,)
    assert np.array_equal(oracle.asf(f, 0), f)
    G, PS = oracle.granulometry(np.zeros((0, 3), np.uint8), 2)
    assert np.array_equal(G, [0, 0, 0])
