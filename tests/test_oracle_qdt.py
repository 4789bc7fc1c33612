"""Pins of the oracle's quasi-distance transform (Eq. 13-15, Algorithm 6)
against things other than the oracle:

- binary images: the distance d is the chessboard distance to the nearest
  background pixel (brute force over all pixel pairs), the residual is 1 on
  the object, and d is already 1-Lipschitz (no eta step changes it);
- grey images: the erosions eps_s(f) taken directly as (2s+1)^2 window
  minima (scipy.ndimage.grey_erosion with nearest borders, which equals the
  clipped window), never by iterating 3x3 steps; d = 1 + the first s of
  largest residual, r = that residual, and the number of changing erosions;
- the limit of eta: the largest 1-Lipschitz (chessboard) function below d,
  min over q of d(q) + max(|dx|, |dy|), and the number of eta steps that
  change something, from the same brute force.
"""
import numpy as np
import pytest
from scipy import ndimage

import oracle

DTYPES = [np.uint8, np.float32, np.float64]


def chessboard(shape):
    Y, X = shape
    yy, xx = np.mgrid[0:Y, 0:X]
    p = np.stack([yy.ravel(), xx.ravel()], 1)
    return np.maximum(np.abs(p[:, None, 0] - p[None, :, 0]), np.abs(p[:, None, 1] - p[None, :, 1]))


def lipschitz_limit(d):
    """min over q of d(q) + rho(p, q), and the eta step count: the largest,
    over p, of the nearest q attaining that minimum."""
    rho = chessboard(d.shape)
    dv = d.ravel().astype(np.int64)
    cand = dv[None, :] + rho
    lim = cand.min(axis=1)
    n = np.where(cand == lim[:, None], rho, np.iinfo(np.int64).max).min(axis=1)
    return lim.reshape(d.shape), int(n.max()) if n.size else 0


def direct_qdt(f):
    Y, X = f.shape
    S = max(X, Y) + 1
    eros = [f] + [ndimage.grey_erosion(f, size=(2 * s + 1, 2 * s + 1), mode="nearest")
                  for s in range(1, S + 1)]
    wide = np.int64 if f.dtype == np.uint8 else f.dtype
    res = np.stack([eros[s].astype(wide) - eros[s + 1].astype(wide) for s in range(S)])
    r = res.max(axis=0)
    first = res.argmax(axis=0)          # the first s reaching the maximum
    d = np.where(r > 0, first + 1, 0).astype(np.int32)
    changing = [s for s in range(S) if not np.array_equal(eros[s], eros[s + 1])]
    steps = max(changing) + 1 if changing else 0
    assert changing == list(range(steps))   # once stable, stable for good
    return d, r.astype(f.dtype), steps


def binary(shape, seed, frac):
    rng = np.random.default_rng(seed)
    b = (rng.random(shape) < frac).astype(np.uint8)
    b = ndimage.binary_dilation(b, iterations=2).astype(np.uint8)   # blobs
    return b


@pytest.mark.parametrize("shape,seed", [((1, 12), 0), ((9, 1), 1), ((14, 17), 2), ((25, 21), 3)])
def test_binary_image_gives_chessboard_distance(shape, seed):
    obj = 1 - binary(shape, seed, 0.08)      # objects with background blobs
    if obj.all():
        obj[0, 0] = 0
    rho = chessboard(shape)
    bg = (obj.ravel() == 0)
    dist = np.where(obj.ravel() == 1, rho[:, bg].min(axis=1), 0).reshape(shape)
    for dtype in DTYPES:
        f = obj.astype(dtype)
        dl1, d, r, steps, eta = oracle.quasi_distance(f)
        assert np.array_equal(d, dist)
        assert np.array_equal(r, f)
        assert steps == dist.max()
        assert np.array_equal(dl1, dist) and eta == 0


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("shape,seed,levels", [((1, 1), 0, 3), ((1, 15), 1, 4), ((12, 1), 2, 4),
                                               ((10, 13), 3, 5), ((19, 16), 4, 9), ((23, 27), 5, 3)])
def test_grey_qdt_matches_direct_erosions(dtype, shape, seed, levels):
    rng = np.random.default_rng(seed)
    v = rng.integers(0, levels, size=shape)
    f = (v * 20).astype(dtype) if dtype == np.uint8 else (v * 0.3 - 0.5).astype(dtype)
    dl1, d, r, steps, eta = oracle.quasi_distance(f)
    ed, er, esteps = direct_qdt(f)
    assert np.array_equal(d, ed)
    assert np.array_equal(r, er)
    assert steps == esteps
    lim, n = lipschitz_limit(d)
    assert np.array_equal(dl1, lim)
    assert eta == n


def test_first_of_equal_residuals_wins():
    # a ramp: at its top end every erosion removes exactly 1, so the first
    # erosion already reaches the largest residual
    f = np.arange(6, dtype=np.uint8)[None, :]
    dl1, d, r, steps, eta = oracle.quasi_distance(f)
    assert np.array_equal(r, [[0, 1, 1, 1, 1, 1]])
    assert np.array_equal(d, [[0, 1, 1, 1, 1, 1]])
    assert steps == 5
    assert np.array_equal(dl1, d) and eta == 0


def test_eta_lowers_steep_distances():
    # A deep pit Z (0) at x = 0, a pit of 50 at x = 5 and a 75 at x = 8 on a
    # plateau of 100.  Pixel 6 drops 100 -> 50 at the first erosion (residual
    # 50, the largest, so d = 1).  Its neighbour 7 first drops 100 -> 75 and
    # then 75 -> 50 (residuals 25) and only reaches a residual of 50 when Z
    # arrives at erosion 7, so d jumps from 1 to 7; eta caps it at 2 and the
    # plateau to its right follows at 3, 4, 5, 6 (five eta steps).
    row = np.array([0, 100, 100, 100, 100, 50, 100, 100, 75, 100, 100, 100], np.uint8)
    f = np.repeat(row[None, :], 3, axis=0)
    dl1, d, r, steps, eta = oracle.quasi_distance(f)
    for y in range(3):
        assert np.array_equal(d[y], [0, 1, 2, 2, 1, 5, 1, 7, 8, 9, 10, 11])
        assert np.array_equal(r[y], [0, 100, 100] + [50] * 9)
        assert np.array_equal(dl1[y], [0, 1, 2, 2, 1, 2, 1, 2, 3, 4, 5, 6])
    assert steps == 11 and eta == 5
    lim, n = lipschitz_limit(d)
    assert np.array_equal(dl1, lim) and eta == n


def test_constant_and_empty():
    for dtype in DTYPES:
        f = np.full((5, 8), 3, dtype=dtype)
        dl1, d, r, steps, eta = oracle.quasi_distance(f)
        assert not dl1.any() and not d.any() and not r.any() and steps == 0 and eta == 0
    dl1, d, r, steps, eta = oracle.quasi_distance(np.zeros((0, 4), np.float32))
    assert dl1.shape == (0, 4) and steps == 0 and eta == 0
