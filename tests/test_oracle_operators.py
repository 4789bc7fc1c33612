"""Pins of the oracle's reconstruction-based operators (Section 2, Eq. 6-12)
against things other than the oracle itself:

- an independent reconstruction: a priority flood over 8-connected paths
  (a pixel's value is the best bottleneck over all paths from the marker,
  the widest-path characterisation of geodesic reconstruction), written
  here with heapq and no iteration of 3x3 steps;
- closed forms on constructed images: isolated plateaus (H-maxima lowers a
  dome of contrast c to max(c - h, 0) above its surroundings), closed and
  leaking rings (hole filling), objects touching and not touching the
  border, and squares that an erosion of size s keeps or deletes;
- scipy.ndimage.grey_erosion (edge replication equals the clipped window)
  for the marker of the opening by reconstruction;
- invariants: HFILL >= f and equals f on the border, RAOBJ is 0 on the
  border, 0 <= DOME <= h on uint8, idempotence.
"""
import heapq

import numpy as np
import pytest
from scipy import ndimage

import oracle

DTYPES = [np.uint8, np.float32, np.float64]
NEIGH = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1) if (dy, dx) != (0, 0)]


def flood_rec_dilation(g, f):
    """Reconstruction by dilation of g under f for g <= f: each pixel gets
    the largest value v such that some pixel q with g(q) >= v reaches it
    through 8-connected pixels whose f is >= v (a max-heap flood)."""
    g = np.asarray(g, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    assert np.all(g <= f)
    Y, X = f.shape
    best = g.copy()
    done = np.zeros((Y, X), dtype=bool)
    heap = [(-best[y, x], y, x) for y in range(Y) for x in range(X)]
    heapq.heapify(heap)
    while heap:
        nv, y, x = heapq.heappop(heap)
        if done[y, x]:
            continue
        done[y, x] = True
        v = -nv
        for dy, dx in NEIGH:
            yy, xx = y + dy, x + dx
            if 0 <= yy < Y and 0 <= xx < X and not done[yy, xx]:
                cand = min(v, f[yy, xx])
                if cand > best[yy, xx]:
                    best[yy, xx] = cand
                    heapq.heappush(heap, (-cand, yy, xx))
    return best


def flood_rec_erosion(g, f):
    """Reconstruction by erosion of g above f (g >= f), by negation."""
    return -flood_rec_dilation(-np.asarray(g, dtype=np.float64), -np.asarray(f, dtype=np.float64))


def rand_img(shape, dtype, seed, levels):
    rng = np.random.default_rng(seed)
    v = rng.integers(0, levels, size=shape)
    if np.dtype(dtype) == np.uint8:
        return (v * (255 // (levels - 1))).astype(np.uint8)
    return (v.astype(np.float64) * 0.37 - 1.1).astype(dtype)


def border_frame(f, inner):
    m = np.full(f.shape, inner, dtype=np.float64)
    m[0, :], m[-1, :], m[:, 0], m[:, -1] = f[0, :], f[-1, :], f[:, 0], f[:, -1]
    return m


SHAPES = [(1, 1), (1, 11), (9, 1), (2, 2), (13, 17), (24, 19)]


# ---------------------------------------------------------------------------
# against the independent flood
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("shape", SHAPES)
def test_hmax_and_dome_match_flood(dtype, shape):
    f = rand_img(shape, dtype, seed=shape[0] * 31 + shape[1], levels=7)
    h = 2 * (255 // 6) if dtype == np.uint8 else 0.8
    if dtype == np.uint8:
        marker = np.clip(f.astype(np.int64) - h, 0, 255)
    else:
        marker = (f - np.dtype(dtype).type(h)).astype(np.float64)
    expect = flood_rec_dilation(marker, f).astype(dtype)
    got, steps, conv = oracle.hmax(f, h)
    assert conv
    assert np.array_equal(got, expect)
    d, steps_d, _ = oracle.dome(f, h)
    assert steps_d == steps
    if dtype == np.uint8:
        assert np.array_equal(d, (f.astype(np.int64) - expect.astype(np.int64)).astype(np.uint8))
    else:
        assert np.array_equal(d, f - expect)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("shape", SHAPES)
def test_hfill_matches_flood(dtype, shape):
    f = rand_img(shape, dtype, seed=shape[0] + 7 * shape[1], levels=5)
    expect = flood_rec_erosion(border_frame(f, f.max()), f).astype(dtype)
    got, _, conv = oracle.hfill(f)
    assert conv and np.array_equal(got, expect)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("shape", SHAPES)
def test_raobj_matches_flood(dtype, shape):
    f = rand_img(shape, dtype, seed=shape[0] * 3 + shape[1], levels=5)
    rec = flood_rec_dilation(border_frame(f, f.min()), f).astype(dtype)
    got, _, conv = oracle.raobj(f)
    assert conv
    if dtype == np.uint8:
        assert np.array_equal(got, (f.astype(np.int64) - rec.astype(np.int64)).astype(np.uint8))
    else:
        assert np.array_equal(got, f - rec)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("s", [0, 1, 2, 4])
def test_open_by_reconstruction_matches_scipy_and_flood(dtype, s):
    f = rand_img((21, 26), dtype, seed=40 + s, levels=6)
    eroded = ndimage.grey_erosion(f, size=(2 * s + 1, 2 * s + 1), mode="nearest")
    expect = flood_rec_dilation(eroded, f).astype(dtype)
    got, _, conv = oracle.open_by_reconstruction(f, s)
    assert conv and np.array_equal(got, expect)


# ---------------------------------------------------------------------------
# closed forms on constructed images
# ---------------------------------------------------------------------------
def plateaus(dtype):
    """Background 10, a dome A of 60 (contrast 50) and a dome B of 25
    (contrast 15), apart from each other and from the border."""
    f = np.full((20, 30), 10, dtype=dtype)
    f[3:8, 4:10] = 60
    f[12:17, 18:27] = 25
    return f


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("h", [0, 5, 15, 30, 50, 70, 300])
def test_hmax_on_isolated_plateaus(dtype, h):
    f = plateaus(dtype)
    got, _, conv = oracle.hmax(f, h)
    assert conv
    # rec(p) = max over q of min(f(q) - h, lowest f on a path q -> p): the
    # background gets max(10 - h, min(60 - h, 10)), dome A keeps 60 - h and
    # dome B gets max(25 - h, min(60 - h, 10)).  Up to h = 50 domes of
    # contrast c keep max(c - h, 0) above the background of 10; beyond it the
    # whole image flattens at 60 - h (0 once uint8 saturates).
    if h <= 50:
        expect = np.full_like(f, 10)
        expect[3:8, 4:10] = 60 - h
        expect[12:17, 18:27] = 10 + max(15 - h, 0)
    else:
        expect = np.full_like(f, max(60 - h, 0) if dtype == np.uint8 else 60 - h)
    assert np.array_equal(got, expect), (h, np.unique(got))


@pytest.mark.parametrize("dtype", DTYPES)
def test_dome_is_capped_contrast(dtype):
    f = plateaus(dtype)
    for h in (5, 15, 30, 50):
        d, _, _ = oracle.dome(f, h)
        expect = np.zeros_like(f)
        expect[3:8, 4:10] = min(50, h)
        expect[12:17, 18:27] = min(15, h)
        assert np.array_equal(d, expect), h


def test_hmax_uint8_marker_saturates():
    f = np.array([[0, 3, 200], [1, 250, 2]], dtype=np.uint8)
    got, _, _ = oracle.hmax(f, 100)
    # marker max(f - 100, 0) = [[0,0,100],[0,150,0]]; every pixel neighbours
    # the 150, so each becomes min(150, f)
    assert np.array_equal(got, np.minimum(f, 150).astype(np.uint8))
    assert np.array_equal(oracle.hmax(f, 255)[0], np.zeros_like(f))
    assert np.array_equal(oracle.hmax(f, 1000)[0], np.zeros_like(f))
    assert np.array_equal(oracle.hmax(f, 0)[0], f)
    with pytest.raises(ValueError):
        oracle.hmax(f, 1.5)
    with pytest.raises(ValueError):
        oracle.hmax(f, -1)


def ring_image(dtype, gap=None):
    """Background 100 reaching the border, a ring of 200 around a hole of
    50; gap = value of one ring pixel (a leak) or None."""
    f = np.full((15, 16), 100, dtype=dtype)
    f[3:12, 4:13] = 200
    f[4:11, 5:12] = 50
    if gap is not None:
        f[3, 8] = gap
    return f


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("gap,fill", [(None, 200), (120, 120), (70, 100), (30, 100)])
def test_hfill_fills_enclosed_hole_to_its_spill_level(dtype, gap, fill):
    f = ring_image(dtype, gap)
    got, _, conv = oracle.hfill(f)
    assert conv
    expect = f.copy()
    expect[4:11, 5:12] = fill
    if gap is not None and gap < fill:
        expect[3, 8] = fill       # the gap itself lies in the basin
    assert np.array_equal(got, expect)


@pytest.mark.parametrize("dtype", DTYPES)
def test_raobj_removes_only_border_objects(dtype):
    f = np.zeros((18, 22), dtype=dtype)
    f[0:5, 3:8] = 90           # touches the top border
    f[8:12, 9:14] = 70         # interior object
    f[13:18, 15:22] = 40       # touches the bottom-right corner
    f[15, 18] = 80             # with a peak inside
    f[2, 15] = 55              # a single interior pixel
    got, _, conv = oracle.raobj(f)
    assert conv
    expect = np.zeros_like(f)
    expect[8:12, 9:14] = 70
    expect[2, 15] = 55
    # grey-level: the border object reconstructs only up to the level that
    # connects it to the border (40), so its inner peak keeps 80 - 40
    expect[15, 18] = 40
    assert np.array_equal(got, expect)


def squares(dtype):
    """Squares of sides 3, 5 and 9 away from the border; corner squares of
    sides 2 and 3."""
    f = np.zeros((30, 40), dtype=dtype)
    f[5:8, 5:8] = 1
    f[5:10, 15:20] = 1
    f[15:24, 5:14] = 1
    f[0:2, 38:40] = 1
    f[27:30, 0:3] = 1
    return f


@pytest.mark.parametrize("dtype", DTYPES)
def test_opening_by_reconstruction_keeps_squares_that_survive_erosion(dtype):
    f = squares(dtype)
    got, _, _ = oracle.open_by_reconstruction(f, 2)
    # a 5x5 erosion (s = 2) deletes the interior 3x3 square, keeps one
    # pixel of the 5x5 square and a 5x5 core of the 9x9 one; the window is
    # clipped to the image, so a corner square survives when its side is at
    # least s + 1 (3 survives, 2 does not).  The reconstruction restores
    # every surviving square in full.
    expect = f.copy()
    expect[5:8, 5:8] = 0
    expect[0:2, 38:40] = 0
    assert np.array_equal(got, expect)
    assert np.array_equal(oracle.open_by_reconstruction(f, 0)[0], f)
    assert not oracle.open_by_reconstruction(f, 5)[0].any()


# ---------------------------------------------------------------------------
# invariants, special cases
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", DTYPES)
def test_operator_invariants(dtype):
    f = rand_img((23, 29), dtype, seed=5, levels=9)
    fill, _, _ = oracle.hfill(f)
    assert np.all(fill >= f)
    for edge in (np.s_[0, :], np.s_[-1, :], np.s_[:, 0], np.s_[:, -1]):
        assert np.array_equal(fill[edge], f[edge])
    assert np.array_equal(oracle.hfill(fill)[0], fill)
    ra, _, _ = oracle.raobj(f)
    for edge in (np.s_[0, :], np.s_[-1, :], np.s_[:, 0], np.s_[:, -1]):
        assert not ra[edge].any()
    assert np.all(ra <= f) if dtype == np.uint8 else np.all(ra >= 0)
    op, _, _ = oracle.open_by_reconstruction(f, 2)
    assert np.all(op <= f)
    assert np.array_equal(oracle.open_by_reconstruction(op, 2)[0], op)


def test_dome_bounds_uint8():
    f = rand_img((25, 31), np.uint8, seed=9, levels=12)
    for h in (0, 20, 69, 255):
        d, _, _ = oracle.dome(f, h)
        assert d.max() <= h
        r, _, _ = oracle.hmax(f, h)
        assert np.all(r.astype(int) >= np.maximum(f.astype(int) - h, 0))
        assert np.all(r <= f)


def test_operator_step_cap_forms_from_the_capped_chain():
    f = ring_image(np.uint8, gap=120)
    _, full, conv = oracle.hfill(f)
    assert conv and full > 2
    got, steps, conv = oracle.hfill(f, max_steps=2)
    assert not conv and steps == 2
    m = border_frame(f, f.max()).astype(np.uint8)
    assert np.array_equal(got, oracle.chain(oracle.ERODE, m, 2, f))


def test_operators_on_empty_images():
    e = np.zeros((0, 5), dtype=np.float32)
    for fn in (lambda x: oracle.hmax(x, 1.0), lambda x: oracle.dome(x, 1.0), oracle.hfill,
               oracle.raobj, lambda x: oracle.open_by_reconstruction(x, 3)):
        out, steps, conv = fn(e)
        assert out.shape == (0, 5) and steps == 0 and conv
