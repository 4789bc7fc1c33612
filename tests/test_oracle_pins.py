"""Pins of the CPU oracle to facts other than itself (no GPU).

Each test checks the oracle against something the paper's definitions or
plain mathematics fix: brute-force window extrema over the clipped square
structuring element (Section 2, Eq. 1-2), the decomposition of the 3x3
square into a row and a column pass (Section 3.1), reconstruction (Eq. 5)
as threshold decomposition with 8-connected flood fill, invariants and
dualities of geodesic operators, special cases with known step counts,
library routines for the plain case, and exact finite differences for the
reference gradient.
"""
import itertools

import numpy as np
import pytest
import torch
from scipy import ndimage

import oracle
import workloads

DTYPES = [np.uint8, np.float32, np.float64]
SHAPES = [(1, 1), (1, 7), (6, 1), (5, 9), (9, 4), (13, 11)]


def rand_img(shape, dtype, seed, levels=None):
    rng = np.random.default_rng(seed)
    if np.dtype(dtype) == np.uint8:
        hi = 256 if levels is None else levels
        return rng.integers(0, hi, size=shape).astype(np.uint8)
    if levels is not None:
        return (rng.integers(0, levels, size=shape) / levels).astype(dtype)
    return rng.standard_normal(shape).astype(dtype)


def brute_window(op, f, n):
    """Extremum over the (2n+1)^2 window clipped to the image, by direct
    enumeration of the window for every pixel."""
    Y, X = f.shape
    out = np.empty_like(f)
    red = np.max if op == oracle.DILATE else np.min
    for y in range(Y):
        for x in range(X):
            out[y, x] = red(f[max(0, y - n):y + n + 1, max(0, x - n):x + n + 1])
    return out


def neutral(op, dtype):
    if np.dtype(dtype) == np.uint8:
        return 0 if op == oracle.DILATE else 255
    return -np.inf if op == oracle.DILATE else np.inf


def top(op, dtype):
    """Value that never wins the clamp (mask >= everything for dilation)."""
    return neutral(oracle.ERODE if op == oracle.DILATE else oracle.DILATE, dtype)


# --------------------------------------------------------------------------
# P1: n chained plain 3x3 steps equal one (2n+1)x(2n+1) clipped window.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("op", [oracle.DILATE, oracle.ERODE])
def test_plain_chain_is_window_extremum(dtype, shape, op):
    f = rand_img(shape, dtype, seed=hash((shape, op)) % 1000)
    for n in (0, 1, 2, 3, 7):
        got = oracle.chain(op, f, n)
        assert got.dtype == f.dtype
        np.testing.assert_array_equal(got, brute_window(op, f, n), err_msg=f"n={n}")


@pytest.mark.parametrize("dtype", DTYPES)
def test_plain_chain_matches_scipy_rank_filter(dtype):
    # Replicated borders leave the clipped window's extremum unchanged, so
    # scipy's 'nearest' mode is the same operator.
    f = rand_img((37, 23), dtype, seed=5)
    for n in (1, 4, 13):
        np.testing.assert_array_equal(
            oracle.chain(oracle.DILATE, f, n),
            ndimage.maximum_filter(f, size=2 * n + 1, mode="nearest"))
        np.testing.assert_array_equal(
            oracle.chain(oracle.ERODE, f, n),
            ndimage.minimum_filter(f, size=2 * n + 1, mode="nearest"))


# --------------------------------------------------------------------------
# P2: SE decomposition, eps_1 = eps_1^x o eps_1^y = eps_1^y o eps_1^x.
# --------------------------------------------------------------------------
def row_pass(op, f):
    red = np.maximum if op == oracle.DILATE else np.minimum
    g = f.copy()
    g[:, 1:] = red(g[:, 1:], f[:, :-1])
    g[:, :-1] = red(g[:, :-1], f[:, 1:])
    return g


def col_pass(op, f):
    return row_pass(op, f.T).T


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("op", [oracle.DILATE, oracle.ERODE])
def test_step_is_row_then_column_pass(dtype, op):
    f = rand_img((17, 29), dtype, seed=11)
    one = oracle.step(op, f)
    np.testing.assert_array_equal(one, col_pass(op, row_pass(op, f)))
    np.testing.assert_array_equal(one, row_pass(op, col_pass(op, f)))


# --------------------------------------------------------------------------
# Geodesic step: Eq. 3 and its dual, on small images with many ties.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", DTYPES)
def test_geodesic_step_definition(dtype):
    f = rand_img((9, 14), dtype, seed=21, levels=6)
    m = rand_img((9, 14), dtype, seed=22, levels=6)
    np.testing.assert_array_equal(oracle.step(oracle.DILATE, f, m),
                                  np.minimum(brute_window(oracle.DILATE, f, 1), m))
    np.testing.assert_array_equal(oracle.step(oracle.ERODE, f, m),
                                  np.maximum(brute_window(oracle.ERODE, f, 1), m))


# --------------------------------------------------------------------------
# P3: reconstruction as threshold decomposition + 8-connected flood fill.
# --------------------------------------------------------------------------
EIGHT = np.ones((3, 3), dtype=bool)


def flood_reconstruct_dilation(f, m):
    """rec(p) = max{t : p lies in a component of {m >= t} meeting {f >= t}}."""
    assert np.all(f <= m)
    levels = np.unique(np.concatenate([f.ravel(), m.ravel()]))
    rec = np.full(f.shape, levels[0], dtype=f.dtype)
    for t in levels:
        lab, _ = ndimage.label(m >= t, structure=EIGHT)
        seeds = np.unique(lab[(f >= t) & (lab > 0)])
        reached = np.isin(lab, seeds) & (lab > 0)
        rec[reached] = t
    return rec


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("shape", [(1, 9), (8, 1), (12, 12), (17, 23), (31, 20)])
def test_reconstruction_by_dilation_is_flood_fill(dtype, shape):
    for seed in range(3):
        m = rand_img(shape, dtype, seed=100 + seed, levels=7)
        f = np.minimum(m, rand_img(shape, dtype, seed=200 + seed, levels=7))
        # sparse marker: most pixels at the lowest level
        keep = np.random.default_rng(seed).random(shape) < 0.1
        f = np.where(keep, f, np.zeros_like(f) if dtype == np.uint8 else np.full_like(f, -1.0))
        f = np.minimum(f, m)
        rec, steps, conv = oracle.reconstruct(oracle.DILATE, f, m)
        assert conv
        np.testing.assert_array_equal(rec, flood_reconstruct_dilation(f, m))


@pytest.mark.parametrize("dtype", DTYPES)
def test_reconstruction_by_erosion_is_dual_flood_fill(dtype):
    shape = (19, 14)
    m = rand_img(shape, dtype, seed=7, levels=6)
    f = np.maximum(m, rand_img(shape, dtype, seed=8, levels=6))
    rec, _, conv = oracle.reconstruct(oracle.ERODE, f, m)
    assert conv
    if dtype == np.uint8:
        expect = 255 - flood_reconstruct_dilation(255 - f, 255 - m)
    else:
        expect = -flood_reconstruct_dilation(-f, -m)
    np.testing.assert_array_equal(rec, expect)


# --------------------------------------------------------------------------
# P4: invariants.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", DTYPES)
def test_geodesic_invariants(dtype):
    shape = (16, 21)
    m = rand_img(shape, dtype, seed=31, levels=20)
    f = np.minimum(m, rand_img(shape, dtype, seed=32, levels=20))
    prev = f
    chains = [f]
    for n in range(1, 9):
        cur = oracle.chain(oracle.DILATE, f, n, m)
        assert np.all(f <= cur) and np.all(cur <= m)        # marker <= result <= mask
        assert np.all(prev <= cur)                          # monotone in n
        chains.append(cur)
        prev = cur
    for a, b in [(1, 2), (3, 4), (2, 6)]:                   # delta_a o delta_b = delta_{a+b}
        np.testing.assert_array_equal(oracle.chain(oracle.DILATE, chains[b], a, m), chains[a + b])
    rec, steps, conv = oracle.reconstruct(oracle.DILATE, f, m)
    assert conv
    np.testing.assert_array_equal(oracle.chain(oracle.DILATE, f, steps, m), rec)
    np.testing.assert_array_equal(oracle.chain(oracle.DILATE, f, steps + 5, m), rec)
    if steps > 0:  # the last counted step did change something
        assert not np.array_equal(oracle.chain(oracle.DILATE, f, steps - 1, m), rec)
    rec2, steps2, _ = oracle.reconstruct(oracle.DILATE, rec, m)   # idempotence
    np.testing.assert_array_equal(rec2, rec)
    assert steps2 == 0


@pytest.mark.parametrize("dtype", DTYPES)
def test_increasing_in_marker_and_mask(dtype):
    shape = (11, 13)
    m1 = rand_img(shape, dtype, seed=41, levels=9)
    m2 = np.maximum(m1, rand_img(shape, dtype, seed=42, levels=9))
    f1 = np.minimum(m1, rand_img(shape, dtype, seed=43, levels=9))
    f2 = np.minimum(m1, np.maximum(f1, rand_img(shape, dtype, seed=44, levels=9)))
    for n in (1, 3, 6):
        a = oracle.chain(oracle.DILATE, f1, n, m1)
        assert np.all(a <= oracle.chain(oracle.DILATE, f2, n, m1))
        assert np.all(a <= oracle.chain(oracle.DILATE, f1, n, m2))


@pytest.mark.parametrize("dtype", DTYPES)
def test_duality(dtype):
    shape = (14, 9)
    m = rand_img(shape, dtype, seed=51)
    f = rand_img(shape, dtype, seed=52)
    for n in (1, 2, 5):
        e = oracle.chain(oracle.ERODE, f, n, m)
        if dtype == np.uint8:
            d = 255 - oracle.chain(oracle.DILATE, 255 - f, n, 255 - m)
        else:
            d = -oracle.chain(oracle.DILATE, -f, n, -m)
        np.testing.assert_array_equal(e, d)


# --------------------------------------------------------------------------
# P5: special cases.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("op", [oracle.DILATE, oracle.ERODE])
def test_inactive_mask_gives_plain_chain(dtype, op):
    f = rand_img((10, 12), dtype, seed=61)
    m = np.full_like(f, top(op, dtype))
    for n in (1, 4):
        np.testing.assert_array_equal(oracle.chain(op, f, n, m), oracle.chain(op, f, n))


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("op", [oracle.DILATE, oracle.ERODE])
def test_marker_equal_mask_is_fixed_point(dtype, op):
    m = rand_img((9, 8), dtype, seed=62)
    np.testing.assert_array_equal(oracle.chain(op, m, 5, m), m)
    rec, steps, conv = oracle.reconstruct(op, m, m)
    assert conv and steps == 0
    np.testing.assert_array_equal(rec, m)


@pytest.mark.parametrize("shape", [(1, 1), (1, 10), (7, 3), (12, 30), (25, 25)])
def test_corner_seed_in_flat_mask(shape):
    Y, X = shape
    m = np.full(shape, 200, dtype=np.uint8)
    f = np.zeros(shape, dtype=np.uint8)
    f[0, 0] = 200
    rec, steps, conv = oracle.reconstruct(oracle.DILATE, f, m)
    assert conv
    np.testing.assert_array_equal(rec, m)
    assert steps == max(X, Y) - 1   # Chebyshev distance to the far corner


def serpentine(rows, width):
    """Corridor mask: every other row open, joined alternately at the right
    and left ends."""
    Y = 2 * rows - 1
    m = np.zeros((Y, width), dtype=np.uint8)
    for r in range(rows):
        m[2 * r, :] = 1
        if r < rows - 1:
            m[2 * r + 1, width - 1 if r % 2 == 0 else 0] = 1
    return m


def bfs_max_distance(mask, seed):
    """Largest 8-connected geodesic distance from seed inside mask (BFS)."""
    Y, X = mask.shape
    dist = -np.ones(mask.shape, dtype=np.int64)
    dist[seed] = 0
    frontier = [seed]
    while frontier:
        nxt = []
        for (y, x) in frontier:
            for dy, dx in itertools.product((-1, 0, 1), repeat=2):
                yy, xx = y + dy, x + dx
                if 0 <= yy < Y and 0 <= xx < X and mask[yy, xx] and dist[yy, xx] < 0:
                    dist[yy, xx] = dist[y, x] + 1
                    nxt.append((yy, xx))
        frontier = nxt
    return int(dist.max())


@pytest.mark.parametrize("rows,width", [(2, 5), (4, 9), (9, 17)])
def test_serpentine_step_count(rows, width):
    m = serpentine(rows, width)
    f = np.zeros_like(m)
    f[0, 0] = 1
    rec, steps, conv = oracle.reconstruct(oracle.DILATE, f, m)
    assert conv
    np.testing.assert_array_equal(rec, m)
    assert steps == bfs_max_distance(m, (0, 0))
    # Hand count for the 2-row corridor of width 5: along row 0 to x=3
    # (3 moves), diagonally into the joint (4), diagonally back (5), then
    # left along row 2 to x=0 (8).
    if (rows, width) == (2, 5):
        assert steps == 8
    # A cap below the true length reports non-convergence and the chain.
    rec_c, steps_c, conv_c = oracle.reconstruct(oracle.DILATE, f, m, max_steps=steps - 1)
    assert not conv_c and steps_c == steps - 1
    np.testing.assert_array_equal(rec_c, oracle.chain(oracle.DILATE, f, steps - 1, m))


def test_empty_and_zero_steps():
    f = np.zeros((0, 5), dtype=np.uint8)
    assert oracle.chain(oracle.DILATE, f, 3).shape == (0, 5)
    g = rand_img((4, 6), np.float32, seed=3)
    np.testing.assert_array_equal(oracle.chain(oracle.ERODE, g, 0, g + 1), g)


# --------------------------------------------------------------------------
# Codes: the tie rule equals max_pool2d's index convention (first maximum
# in raster order inside the window) for the plain step.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("op", [oracle.DILATE, oracle.ERODE])
def test_codes_match_max_pool_indices(op):
    f = rand_img((15, 22), np.float64, seed=71, levels=4)   # many ties
    _, codes = oracle.chain_codes(op, f, 1)
    t = torch.from_numpy(f if op == oracle.DILATE else -f)[None, None]
    _, idx = torch.nn.functional.max_pool2d(t, 3, stride=1, padding=1, return_indices=True)
    idx = idx[0, 0].numpy()
    Y, X = f.shape
    yy, xx = np.divmod(idx, X)
    gy, gx = np.mgrid[0:Y, 0:X]
    expect = (yy - gy + 1) * 3 + (xx - gx + 1)
    np.testing.assert_array_equal(codes[0], expect)


def test_codes_mask_wins_ties():
    f = np.array([[1.0, 2.0], [3.0, 4.0]])
    m = np.array([[4.0, 9.0], [0.0, 4.0]])
    out, codes = oracle.chain_codes(oracle.DILATE, f, 1, m)
    np.testing.assert_array_equal(out, [[4.0, 4.0], [0.0, 4.0]])
    # D = 4 everywhere (every clipped window holds the whole image); the
    # first maximum of (0,1) is its lower neighbour (dy=1, dx=0) -> code 7.
    np.testing.assert_array_equal(codes[0], [[9, 7], [9, 9]])


# --------------------------------------------------------------------------
# P6: the reference gradient.
# --------------------------------------------------------------------------
def loss(op, f, m, n, g):
    return float(np.sum(g * oracle.chain(op, f, n, m)))


@pytest.mark.parametrize("op", [oracle.DILATE, oracle.ERODE])
@pytest.mark.parametrize("shape,n", [((5, 6), 1), ((6, 5), 3), ((4, 9), 6)])
def test_gradient_exact_finite_differences(op, shape, n):
    # Integer leaves, all distinct, spaced by >= 1; eps = 1/4 and integer
    # upstream gradients keep every sum exact in float64.
    f, m = workloads.tie_free(*shape, seed=hash(shape) % 97)
    if op == oracle.ERODE:
        f, m = m, f
    g = np.random.default_rng(n).integers(-5, 6, size=shape).astype(np.float64)
    gf, gm = oracle.chain_vjp(op, f, m, n, g)
    eps = 0.25
    for leaf, grad in ((f, gf), (m, gm)):
        for idx in np.ndindex(*shape):
            plus = leaf.copy(); plus[idx] += eps
            minus = leaf.copy(); minus[idx] -= eps
            if leaf is f:
                fd = (loss(op, plus, m, n, g) - loss(op, minus, m, n, g)) / (2 * eps)
            else:
                fd = (loss(op, f, plus, n, g) - loss(op, f, minus, n, g)) / (2 * eps)
            assert fd == grad[idx], (idx, fd, grad[idx])


@pytest.mark.parametrize("op", [oracle.DILATE, oracle.ERODE])
def test_gradient_value_identity(op):
    # With all leaves distinct every output is a copy of exactly one leaf, so
    # d(sum g*y)/d leaf = sum of g over the outputs equal to that leaf's value.
    shape, n = (12, 17), 9
    f, m = workloads.tie_free(*shape, seed=5)
    if op == oracle.ERODE:
        f, m = m, f
    g = np.random.default_rng(9).standard_normal(shape)
    y = oracle.chain(op, f, n, m)
    gf, gm = oracle.chain_vjp(op, f, m, n, g)
    for leaf, grad in ((f, gf), (m, gm)):
        expect = np.zeros(shape)
        for idx in np.ndindex(*shape):
            expect[idx] = g[y == leaf[idx]].sum()
        np.testing.assert_allclose(grad, expect, rtol=0, atol=1e-12)
    # Conservation: every unit of upstream gradient lands somewhere.
    assert abs(gf.sum() + gm.sum() - g.sum()) < 1e-9
