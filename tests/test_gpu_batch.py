"""GPU parity of the batched persistent launch (gc_plan_*) against the CPU
oracle, bit-exact per image, including graph replays, uneven sizes and
chain lengths, in-place items, zero-step and empty items, both tile
families, autotuned plans, an image beyond one launch grid, and items that
run to stability (images and step counts against the oracle's
reconstruction)."""
import json

import numpy as np
import pytest
import torch

import oracle
import workloads
import paper_1911_13074_amd as gc
from paper_1911_13074_amd import abi

pytestmark = pytest.mark.gpu

DTYPES = [np.uint8, np.float32, np.float64]


@pytest.fixture(autouse=True)
def _reset():
    yield
    gc.set_tuning(0, -1)
    gc.autotune_clear()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


def rand_img(shape, dtype, rng, levels=12):
    if np.dtype(dtype) == np.uint8:
        return (rng.integers(0, levels, size=shape) * (255 // (levels - 1))).astype(np.uint8)
    return (rng.integers(0, levels, size=shape) - levels / 2).astype(dtype)


def make_batch(dtype, seed, count, lo, hi, n_lo, n_hi):
    rng = np.random.default_rng(seed)
    items = []
    for _ in range(count):
        h = int(rng.integers(lo, hi + 1))
        w = int(rng.integers(lo, hi + 1))
        n = int(rng.integers(n_lo, n_hi + 1))
        items.append((rand_img((h, w), dtype, rng), rand_img((h, w), dtype, rng), n))
    return items


def check_items(op, host_items, outs, geodesic=True):
    code = oracle.DILATE if op == "dilate" else oracle.ERODE
    for i, ((f, m, n), o) in enumerate(zip(host_items, outs)):
        ref = oracle.chain(code, f, n, m if geodesic else None)
        got = host(o)
        assert np.array_equal(got, ref), f"item {i}: shape {f.shape}, n={n}"


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("op", ["dilate", "erode"])
def test_uneven_batch(dtype, op):
    items = make_batch(dtype, seed=11, count=12, lo=1, hi=300, n_lo=1, n_hi=90)
    items.append((items[0][0][:0], items[0][1][:0], 5))          # empty image
    items.append((items[1][0], items[1][1], 0))                   # zero steps
    plan = gc.BatchPlan(op, [(dev(f), dev(m), n) for f, m, n in items])
    plan.launch()
    plan.status()
    check_items(op, items, plan.outs)


@pytest.mark.parametrize("tile,k", [(0, 8), (0, 21), (0, 42), (1, 5), (1, 21), (2, 32), (3, 16), (3, 32), (4, 11)])
def test_launch_shapes(tile, k):
    gc.set_tuning(k, tile)
    items = make_batch(np.uint8, seed=tile * 100 + k, count=6, lo=50, hi=400, n_lo=k, n_hi=3 * k + 7)
    plan = gc.BatchPlan("dilate", [(dev(f), dev(m), n) for f, m, n in items])
    info = plan.info()
    assert info["tile"] == tile
    plan.launch()
    plan.status()
    check_items("dilate", items, plan.outs)


def test_plain_batch_and_in_place():
    rng = np.random.default_rng(5)
    items = [(rand_img((h, w), np.float32, rng, levels=50), None, n)
             for h, w, n in [(200, 33, 7), (64, 64, 32), (1, 500, 13), (257, 129, 91)]]
    ts = [dev(f) for f, _, _ in items]
    plan = gc.BatchPlan("erode", [(t, None, n, t) for t, (_, _, n) in zip(ts, items)])
    plan.launch()
    plan.status()
    for (f, _, n), t in zip(items, ts):
        assert np.array_equal(host(t), oracle.chain(oracle.ERODE, f, n))


def test_in_place_single_block_and_many_blocks():
    rng = np.random.default_rng(8)
    cases = [((90, 120), 3), ((300, 200), 100)]
    host_items, dev_items = [], []
    for shape, n in cases:
        f, m = rand_img(shape, np.uint8, rng), rand_img(shape, np.uint8, rng)
        F = dev(f)
        host_items.append((f, m, n))
        dev_items.append((F, dev(m), n, F))
    plan = gc.BatchPlan("dilate", dev_items)
    plan.launch()
    plan.status()
    check_items("dilate", host_items, [d[0] for d in dev_items])


def test_graph_replays_match_eager():
    items = make_batch(np.uint8, seed=3, count=8, lo=64, hi=600, n_lo=20, n_hi=200)
    dev_items = [(dev(f), dev(m), n) for f, m, n in items]
    plan = gc.BatchPlan("dilate", dev_items)
    eager = [host(gc.geodesic_dilate_chain(F, M, n)) for F, M, n in dev_items]
    for rep in range(3):
        for o in plan.outs:
            o.fill_(7)
        torch.cuda.synchronize()
        plan.launch()
        plan.status()
        for i, o in enumerate(plan.outs):
            assert np.array_equal(host(o), eager[i]), f"replay {rep}, item {i}"
        # some unrelated eager work between replays
        _ = gc.dilate_chain(dev_items[0][0], 3)
        torch.cuda.synchronize()
    check_items("dilate", items[:3], plan.outs[:3])


def test_autotuned_plan():
    tile, k = gc.autotune(torch.uint8, "dilate", True, 256, 256)
    assert 0 <= tile <= 4 and k >= 1
    items = make_batch(np.uint8, seed=21, count=10, lo=129, hi=256, n_lo=30, n_hi=120)
    plan = gc.BatchPlan("dilate", [(dev(f), dev(m), n) for f, m, n in items])
    assert plan.info()["tile"] == tile
    plan.launch()
    plan.status()
    check_items("dilate", items, plan.outs)


def test_imported_tuning_table_steers_the_plan(tmp_path):
    """A table loaded from a file decides a plan like one the autotuner
    filled: records for the items' size class that make tile family 0 the
    fastest, with 24 steps per block, give a plan of that family and block
    length, and its results stay bit-exact."""
    rec = {"dtype": abi.GC_U8, "op": abi.GC_DILATE, "geodesic": 1, "log2_width": 9, "log2_height": 9,
           "best_tile": 0, "k": [24, 16, 20, 16, 16], "rate": [9e12, 1e12, 1e12, 1e12, 1e12]}
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"format": "geochain-autotune", "version": 1,
                                "families": abi.GC_TUNE_FAMILIES, "records": [rec]}))
    gc.autotune_clear()
    gc.autotune_load(path)
    try:
        items = make_batch(np.uint8, seed=23, count=6, lo=257, hi=512, n_lo=30, n_hi=90)
        plan = gc.BatchPlan("dilate", [(dev(f), dev(m), n) for f, m, n in items])
        info = plan.info()
        assert info["tile"] == 0 and info["block_steps"] == 24, info
        plan.launch()
        plan.status()
        check_items("dilate", items, plan.outs)
    finally:
        gc.autotune_clear()


def test_stability_plan_keeps_its_shape_under_a_tuning_table(tmp_path):
    """A plan whose items run to stability keeps the built-in launch shape
    (128x128 regions, 20 steps per block: one change word per block) even
    where the table names another family, and its reconstructions match the
    oracle's, step counts included."""
    rec = {"dtype": abi.GC_U8, "op": abi.GC_DILATE, "geodesic": 1, "log2_width": 9, "log2_height": 9,
           "best_tile": 0, "k": [24, 16, 20, 16, 16], "rate": [9e12, 1e12, 1e12, 1e12, 1e12]}
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"format": "geochain-autotune", "version": 1,
                                "families": abi.GC_TUNE_FAMILIES, "records": [rec]}))
    gc.autotune_clear()
    gc.autotune_load(path)
    try:
        rng = np.random.default_rng(29)
        items = []
        for _ in range(4):
            h, w = int(rng.integers(257, 513)), int(rng.integers(257, 513))
            m = rand_img((h, w), np.uint8, rng)
            items.append((np.minimum(rand_img((h, w), np.uint8, rng), m), m))
        plan = gc.BatchPlan("dilate", [(dev(f), dev(m), -1) for f, m in items])
        info = plan.info()
        assert info["tile"] == 2 and info["block_steps"] == 20, info
        plan.launch()
        plan.status()
        steps = plan.steps()
        for i, ((f, m), o) in enumerate(zip(items, plan.outs)):
            ref, n, conv = oracle.reconstruct(oracle.DILATE, f, m)
            assert conv and steps[i] == n, (i, steps[i], n)
            assert np.array_equal(host(o), ref), i
        plan.close()
    finally:
        gc.autotune_clear()


def test_mixed_plan_rejected():
    a = torch.zeros((10, 10), dtype=torch.uint8, device="cuda")
    with pytest.raises(abi.GeochainError) as ei:
        gc.BatchPlan("dilate", [(a, a.clone(), 3), (a.clone(), None, 3)])
    assert ei.value.status == abi.GC_ERR_UNSUPPORTED


@pytest.fixture(scope="module")
def uneven_workload_outputs():
    """The 64-image uneven batch (sides 128..2048, chains 10..1500) in one
    persistent launch; the outputs, copied to the host."""
    batch = workloads.batch_u8()
    dev_items = [(dev(it.marker), dev(it.mask), it.n_steps) for it in batch.items]
    plan = gc.BatchPlan("dilate", dev_items)
    try:
        plan.launch()
        plan.status()
        outs = [host(o) for o in plan.outs]
    finally:
        plan.close()
    del dev_items
    torch.cuda.empty_cache()
    return batch, outs


@pytest.mark.parametrize("chunk", range(4))
def test_uneven_batch_workload_every_image(uneven_workload_outputs, chunk):
    """Every image of the 64-image uneven batch against the oracle's chain
    (Eq. 4), pixel by pixel: images i with i mod 4 == chunk, so each chunk
    holds a mix of sizes and chain lengths (about 5 s of oracle time on 16
    host threads per chunk)."""
    batch, outs = uneven_workload_outputs
    assert len(outs) == 64
    for i in range(chunk, len(batch.items), 4):
        it = batch.items[i]
        ref = oracle.chain(oracle.DILATE, it.marker, it.n_steps, it.mask)
        assert np.array_equal(outs[i], ref), f"image {i}: {it.mask.shape}, n={it.n_steps}"


def test_tuned_plan_matches_and_leaves_inputs_alone():
    """gc_plan_tune times launch shapes on scratch images, then rebuilds the
    plan: results stay bit-exact, in-place items keep their input until the
    launch, and the tuned plan is never slower than the built-in by more
    than noise."""
    rng = np.random.default_rng(21)
    shapes = [(300, 517), (128, 128), (1, 700), (700, 1), (257, 199)]
    items, refs, keep = [], [], []
    for i, (h, w) in enumerate(shapes):
        m = rng.integers(0, 256, size=(h, w)).astype(np.uint8)
        f = np.minimum(m, rng.integers(0, 256, size=(h, w)).astype(np.uint8))
        n = int(rng.integers(5, 90))
        F, M = torch.from_numpy(f).cuda(), torch.from_numpy(m).cuda()
        if i == 0:
            items.append((F, M, n, F))      # in place
        else:
            items.append((F, M, n))
        keep.append((F, M))
        refs.append(oracle.chain(oracle.DILATE, f, n, m))
    plan = gc.BatchPlan("dilate", items)
    before = keep[0][0].clone()
    ms = plan.tune()
    assert ms > 0
    assert torch.equal(keep[0][0], before)   # tuning never touched the caller's images
    outs = plan.launch()
    plan.status()
    info = plan.info()
    assert info["tile"] in (0, 2, 3, 4) and 1 <= info["block_steps"] <= 28
    for out, ref in zip(outs, refs):
        assert np.array_equal(out.cpu().numpy(), ref)
    plan.close()


def test_plan_with_image_beyond_one_launch_grid():
    """A plan that mixes a 131172 x 131035 u8 image (1.7e10 pixels: 1491 x
    1489 tiles of 88 x 88 cores per block of 20 steps, 4.4 million work items
    over its two blocks) with a small image.  After n steps a pixel depends
    only on the marker and mask within chessboard distance n, so the oracle
    on crops checks sampled pixels of the large output; the small one is
    checked whole."""
    W, H, n = 131172, 131035, 40
    gen = torch.Generator(device="cuda").manual_seed(31)
    F = torch.randint(0, 200, (H, W), dtype=torch.uint8, device="cuda", generator=gen)
    M = torch.randint(50, 256, (H, W), dtype=torch.uint8, device="cuda", generator=gen)
    rng = np.random.default_rng(37)
    f2, m2 = rand_img((300, 411), np.uint8, rng), rand_img((300, 411), np.uint8, rng)
    plan = gc.BatchPlan("dilate", [(F, M, n), (dev(f2), dev(m2), 57)])
    try:
        assert plan.info()["work_items"] > 4_000_000
        plan.launch()
        plan.status()
        out = plan.outs[0]
        torch.cuda.synchronize()
        pts = [(0, 0), (0, W - 1), (H - 1, 0), (H - 1, W - 1), (H // 2, W // 2)]
        pts += [(int(rng.integers(0, H)), int(rng.integers(0, W))) for _ in range(30)]
        for y, x in pts:
            y0, y1 = max(0, y - n), min(H, y + n + 1)
            x0, x1 = max(0, x - n), min(W, x + n + 1)
            ref = oracle.chain(oracle.DILATE, F[y0:y1, x0:x1].cpu().numpy(), n, M[y0:y1, x0:x1].cpu().numpy())
            assert int(out[y, x]) == int(ref[y - y0, x - x0]), (y, x)
        assert np.array_equal(host(plan.outs[1]), oracle.chain(oracle.DILATE, f2, 57, m2))
    finally:
        plan.close()
    del F, M, plan
    torch.cuda.empty_cache()


def _serpentine(h, w):
    """Mask open along every even row, the rows joined alternately at the
    right and the left end; marker: one seed at the corridor's start."""
    m = np.zeros((h, w), np.uint8)
    m[0::2, :] = 255
    for y in range(1, h, 2):
        m[y, w - 1 if (y // 2) % 2 == 0 else 0] = 255
    f = np.zeros_like(m)
    f[0, 0] = 255
    return f, m


def _stability_items(dtype, rng):
    """(marker, mask, n_steps, in_place) host items for a mixed plan."""
    items = []
    for shape in ((200, 300), (97, 131)):
        f, m = rand_img(shape, dtype, rng), rand_img(shape, dtype, rng)
        items.append((np.minimum(f, m), m, -1, False))
    f, m = rand_img((120, 77), dtype, rng), rand_img((120, 77), dtype, rng)
    items.append((np.minimum(f, m), m, -1, True))          # in place
    seed_m = np.full((150, 260), 5, dtype)
    seed_f = np.zeros_like(seed_m)
    seed_f[0, 0] = 5                                         # 259 steps: seven replays
    items.append((seed_f, seed_m, -1, False))
    f, m = _serpentine(31, 64)
    items.append((f.astype(dtype), m.astype(dtype), -1, False))   # about a thousand steps
    f, m = rand_img((64, 90), dtype, rng), rand_img((64, 90), dtype, rng)
    items.append((f, m, 37, False))                          # fixed length
    items.append((f, m, 0, False))
    return items


@pytest.mark.parametrize("op", ["dilate", "erode"])
@pytest.mark.parametrize("dtype", DTYPES)
def test_plan_items_run_to_stability(op, dtype):
    """Run-to-stability items (n_steps < 0) beside fixed-length ones in one
    plan, u8, f32 and f64: every image and every step count equals the
    oracle's (the reconstruction for n < 0, the chain otherwise), across
    replays that retire converged images and continue the others (the
    corridor needs about a thousand steps, many replays of 40)."""
    rng = np.random.default_rng(61)
    host_items = _stability_items(dtype, rng)
    if op == "erode":   # reconstruction by erosion: marker above the mask
        host_items = [(np.maximum(f, m) if n < 0 else f, m, n, ip) for f, m, n, ip in host_items]
        host_items[3] = (np.full((150, 260), 5, dtype), np.zeros((150, 260), dtype), -1, False)
        host_items[3][0][0, 0] = 0
        sf, sm = _serpentine(31, 64)
        host_items[4] = ((255 - sf).astype(dtype), (255 - sm).astype(dtype), -1, False)
    code = oracle.DILATE if op == "dilate" else oracle.ERODE
    dev_items = []
    for f, m, n, ip in host_items:
        F, M = dev(f), dev(m)
        dev_items.append((F, M, n, F) if ip else (F, M, n))
    plan = gc.BatchPlan(op, dev_items)
    try:
        plan.launch()
        plan.status()
        steps = plan.steps()
        for i, ((f, m, n, ip), o) in enumerate(zip(host_items, plan.outs)):
            if n < 0:
                ref, ref_steps, conv = oracle.reconstruct(code, f, m)
                assert conv and steps[i] == ref_steps, (i, steps[i], ref_steps)
            else:
                ref = oracle.chain(code, f, n, m)
                assert steps[i] == n
            assert np.array_equal(host(o), ref), f"item {i}: {f.shape} n={n} in_place={ip}"
        assert max(steps) > 160       # at least one image needed several replays
    finally:
        plan.close()


def test_plan_relaunch_and_refusals():
    """A run-to-stability plan launched twice gives the same result (each
    launch starts from the markers); plain items cannot run to stability;
    such plans keep the built-in launch shape."""
    rng = np.random.default_rng(71)
    f, m = rand_img((140, 210), np.uint8, rng), rand_img((140, 210), np.uint8, rng)
    F, M = dev(np.minimum(f, m)), dev(m)
    plan = gc.BatchPlan("dilate", [(F, M, -1)])
    try:
        assert plan.steps() == [-1]      # not launched yet
        plan.launch()
        first = plan.outs[0].clone()
        s1 = plan.steps()
        plan.launch()
        assert torch.equal(plan.outs[0], first) and plan.steps() == s1
        ref, ref_steps, _ = oracle.reconstruct(oracle.DILATE, np.minimum(f, m), m)
        assert np.array_equal(host(first), ref) and s1 == [ref_steps]
        with pytest.raises(gc.GeochainError):
            plan.tune()
    finally:
        plan.close()
    with pytest.raises(gc.GeochainError):
        gc.BatchPlan("dilate", [(F, None, -1)])


@pytest.fixture
def plan_grid(monkeypatch):
    """Sets the grid of plans built inside the test (GEOCHAIN_PLAN_GRID)."""
    def set_grid(n):
        monkeypatch.setenv("GEOCHAIN_PLAN_GRID", str(n))
    yield set_grid
    monkeypatch.delenv("GEOCHAIN_PLAN_GRID", raising=False)


@pytest.mark.parametrize("grid", [1, 3, 4096])
def test_any_grid_finishes(plan_grid, grid):
    """Items are drawn in list order, so the launch finishes whatever part
    of its grid is resident: one workgroup doing everything, three, or 4096
    workgroups (eight times what fits on the device at once, so most of them
    start only after others have left)."""
    plan_grid(grid)
    items = make_batch(np.uint8, seed=40 + grid, count=7, lo=60, hi=420, n_lo=15, n_hi=140)
    plan = gc.BatchPlan("dilate", [(dev(f), dev(m), n) for f, m, n in items])
    assert plan.info()["workgroups"] == grid
    plan.launch()
    plan.status()
    check_items("dilate", items, plan.outs)


def test_two_plans_at_the_same_time():
    """Two plans, each with a grid of all the workgroups the device holds,
    replayed at the same time on two streams: they compete for the CUs, and
    both finish with exact results."""
    a_items = make_batch(np.uint8, seed=51, count=9, lo=100, hi=700, n_lo=40, n_hi=300)
    b_items = make_batch(np.float32, seed=52, count=6, lo=100, hi=500, n_lo=30, n_hi=200)
    plan_a = gc.BatchPlan("dilate", [(dev(f), dev(m), n) for f, m, n in a_items])
    plan_b = gc.BatchPlan("erode", [(dev(f), dev(m), n) for f, m, n in b_items])
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    for _ in range(2):
        with torch.cuda.stream(s1):
            plan_a.launch()
        with torch.cuda.stream(s2):
            plan_b.launch()
    plan_a.status()
    plan_b.status()
    check_items("dilate", a_items, plan_a.outs)
    check_items("erode", b_items, plan_b.outs)


def test_wait_bound_reports_and_drains(monkeypatch):
    """A plan whose dependency waits are bounded at zero (test hook
    GEOCHAIN_PLAN_WAIT_TICKS=0: every wait fails at once): the launch still
    drains, gc_plan_status reports GC_ERR_HIP, and a plan built afterwards
    without the hook is exact again."""
    items = make_batch(np.uint8, seed=61, count=4, lo=200, hi=400, n_lo=60, n_hi=120)
    dev_items = [(dev(f), dev(m), n) for f, m, n in items]
    monkeypatch.setenv("GEOCHAIN_PLAN_WAIT_TICKS", "0")
    bad = gc.BatchPlan("dilate", dev_items)
    monkeypatch.delenv("GEOCHAIN_PLAN_WAIT_TICKS")
    bad.launch()
    with pytest.raises(abi.GeochainError) as ei:
        bad.status()
    assert ei.value.status == abi.GC_ERR_HIP and "bound" in str(ei.value)
    bad.close()
    good = gc.BatchPlan("dilate", dev_items)
    good.launch()
    good.status()
    check_items("dilate", items, good.outs)
