"""GPU parity of the reconstruction-based operators (Eq. 6-12) through the C
ABI against the oracle: bit-exact images (u8 saturating and float
differences are single rounded operations on both sides) and identical
reconstruction step counts, on ragged shapes, rows that are and are not
16-byte aligned (vector and scalar pixel passes), the step cap, h at its
extremes, and the full-size 1024 x 1024 u8 workloads the benchmark times."""
import numpy as np
import pytest
import torch

import oracle
import workloads
import paper_1911_13074_amd as gc
from paper_1911_13074_amd import abi

pytestmark = pytest.mark.gpu

DTYPES = [np.uint8, np.float32, np.float64]
SHAPES = [(1, 1), (1, 300), (300, 1), (2, 2), (67, 129), (200, 517), (513, 385)]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def assert_same(got, expect, what=""):
    assert got.dtype == expect.dtype, what
    if not np.array_equal(got, expect):
        bad = np.argwhere(got != expect)
        y, x = bad[0]
        raise AssertionError(f"{what}: {len(bad)} pixels differ, first at (y={y}, x={x}): "
                             f"got {got[y, x]!r} expected {expect[y, x]!r}")


def levels_img(shape, dtype, seed, levels):
    rng = np.random.default_rng(seed)
    v = rng.integers(0, levels, size=shape)
    if np.dtype(dtype) == np.uint8:
        return (v * (255 // (levels - 1))).astype(np.uint8)
    return (v * 0.37 - 1.1).astype(dtype)


def smooth_img(shape, dtype, seed):
    f = workloads.blur(shape[0], shape[1], 3.0, seed) if min(shape) > 1 else \
        np.random.default_rng(seed).integers(0, 256, size=shape).astype(np.uint8)
    if np.dtype(dtype) == np.uint8:
        return f
    return (f.astype(np.float64) / 255.0 * 3.0 - 1.0).astype(dtype)


def h_for(dtype):
    return 40 if np.dtype(dtype) == np.uint8 else 0.45


OPS = {
    "hmax": (lambda f, **kw: gc.hmax(f, kw.pop("h"), **kw), lambda f, **kw: oracle.hmax(f, kw.pop("h"), **kw)),
    "dome": (lambda f, **kw: gc.dome(f, kw.pop("h"), **kw), lambda f, **kw: oracle.dome(f, kw.pop("h"), **kw)),
    "hfill": (lambda f, **kw: gc.hfill(f, **kw), lambda f, **kw: oracle.hfill(f, **kw)),
    "raobj": (lambda f, **kw: gc.raobj(f, **kw), lambda f, **kw: oracle.raobj(f, **kw)),
    "open_rec": (lambda f, **kw: gc.open_by_reconstruction(f, kw.pop("s"), **kw),
                 lambda f, **kw: oracle.open_by_reconstruction(f, kw.pop("s"), **kw)),
}


def params(name, dtype):
    if name in ("hmax", "dome"):
        return {"h": h_for(dtype)}
    if name == "open_rec":
        return {"s": 3}
    return {}


def check(name, f, what, **extra):
    gpu_fn, ref_fn = OPS[name]
    kw = params(name, f.dtype)
    kw.update(extra)
    out, steps, conv = gpu_fn(dev(f), **dict(kw))
    ref, ref_steps, ref_conv = ref_fn(f, **dict(kw))
    assert conv == ref_conv, what
    assert steps == ref_steps, (what, steps, ref_steps)
    assert_same(host(out), ref, what)
    return steps


@pytest.mark.parametrize("name", list(OPS))
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("shape", SHAPES)
def test_operator_parity(name, dtype, shape):
    check(name, levels_img(shape, dtype, seed=shape[0] * 13 + shape[1], levels=6), f"{name} levels")
    check(name, smooth_img(shape, dtype, seed=shape[0] + shape[1]), f"{name} smooth")


@pytest.mark.parametrize("name", list(OPS))
@pytest.mark.parametrize("dtype", DTYPES)
def test_unaligned_rows_take_the_scalar_pass(name, dtype):
    # a view starting one element into a padded buffer: row starts are not
    # 16-byte aligned, so the pixel passes run one element per lane
    h, w = 150, 203
    f = smooth_img((h, w), dtype, seed=5)
    F = torch.zeros((h, 256), dtype=dev(f).dtype, device="cuda")
    F[:, 1:w + 1] = dev(f)
    fv = F[:, 1:w + 1]
    O = torch.full_like(F, 7)
    ov = O[:, 1:w + 1]
    gpu_fn, ref_fn = OPS[name]
    kw = params(name, f.dtype)
    out, steps, conv = gpu_fn(fv, out=ov, **dict(kw))
    ref, ref_steps, _ = ref_fn(f, **dict(kw))
    assert conv and steps == ref_steps
    assert_same(host(ov), ref, name)
    # nothing outside the view was written
    O = host(O)
    assert (O[:, 0] == 7).all() and (O[:, w + 1:] == 7).all()


@pytest.mark.parametrize("dtype", DTYPES)
def test_hmax_extreme_h(dtype):
    f = smooth_img((90, 140), dtype, seed=11)
    hs = [0, 1, 255, 300, 1000] if dtype == np.uint8 else [0.0, 1e-6, 2.5, 1e30]
    for h in hs:
        check("hmax", f, f"h={h}", h=h)
        check("dome", f, f"h={h}", h=h)


@pytest.mark.parametrize("s", [0, 1, 7, 40])
def test_open_by_reconstruction_sizes(s):
    f = smooth_img((180, 230), np.uint8, seed=s)
    check("open_rec", f, f"s={s}", s=s)


@pytest.mark.parametrize("name", list(OPS))
def test_step_cap(name):
    f = smooth_img((120, 333), np.float32, seed=3)
    full = check(name, f, "uncapped")
    if full < 3:
        pytest.skip("reconstruction too short to cap")
    cap = full // 2
    out, steps, conv = OPS[name][0](dev(f), max_steps=cap, allow_not_converged=True,
                                    **params(name, f.dtype))
    ref, ref_steps, ref_conv = OPS[name][1](f, max_steps=cap, **params(name, f.dtype))
    assert not conv and not ref_conv and steps == ref_steps == cap
    assert_same(host(out), ref, f"{name} capped")
    with pytest.raises(abi.GeochainError) as ei:
        OPS[name][0](dev(f), max_steps=cap, **params(name, f.dtype))
    assert ei.value.status == abi.GC_ERR_NOT_CONVERGED


def test_out_must_not_alias_f():
    F = dev(smooth_img((40, 50), np.uint8, seed=1))
    with pytest.raises(abi.GeochainError) as ei:
        gc.hfill(F, out=F)
    assert ei.value.status == abi.GC_ERR_ALIAS


def test_empty_images():
    e = torch.empty((0, 9), dtype=torch.float32, device="cuda")
    for name in OPS:
        out, steps, conv = OPS[name][0](e, **params(name, np.float32))
        assert out.shape == (0, 9) and steps == 0 and conv


# ---------------------------------------------------------------------------
# full-size workloads (the configuration the benchmark times)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name,extra", [("hmax", {}), ("dome", {}), ("hfill", {}), ("raobj", {}),
                                        ("open_rec", {"s": 5}), ("open_rec", {"s": 75})])
def test_full_size_u8_operators(name, extra):
    f = workloads.operator_u8()
    steps = check(name, f, f"{name} 1024x1024", **extra)
    assert steps > 0
