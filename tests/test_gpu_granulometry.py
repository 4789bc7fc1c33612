"""GPU parity of the granulometry, pattern spectrum and ASF (Eq. 16-20)
through the C ABI against the oracle.  The ASF only selects values, so it is
bit-exact.  G_s sums in float64 on both sides but in different orders: for
u8 images every partial sum is an integer below 2^53, so G and PS are
exact; for float images they agree within the bound of recursive float64
summation, n * 2^-53 * sum|f| (n = pixel count), stated per test below."""
import numpy as np
import pytest
import torch

import oracle
import workloads
import paper_1911_13074_amd as gc

pytestmark = pytest.mark.gpu

DTYPES = [np.uint8, np.float32, np.float64]
SHAPES = [(1, 1), (1, 300), (300, 1), (67, 129), (200, 517), (513, 385)]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def image(shape, dtype, seed):
    f = workloads.blur(shape[0], shape[1], 2.0, seed) if min(shape) > 1 else \
        np.random.default_rng(seed).integers(0, 256, size=shape).astype(np.uint8)
    return f if dtype == np.uint8 else (f / 255.0 * 2.0 - 0.5).astype(dtype)


def check_granulometry(f, s_max, what):
    G, PS = gc.granulometry(dev(f), s_max)
    rG, rPS = oracle.granulometry(f, s_max)
    if f.dtype == np.uint8:
        assert G == list(rG), what
        assert PS == list(rPS), what
    else:
        tol = f.size * 2.0 ** -53 * float(np.abs(f.astype(np.float64)).sum())
        np.testing.assert_allclose(G, rG, rtol=0, atol=tol, err_msg=what)
        np.testing.assert_allclose(PS, rPS, rtol=0, atol=2 * tol, err_msg=what)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("shape", SHAPES)
def test_granulometry_parity(dtype, shape):
    check_granulometry(image(shape, dtype, seed=shape[0] + 3 * shape[1]), 6, f"{shape}")


# 63, 64 and 130 cross the batches in which the per-size sums are added
# (64 sizes per launch)
@pytest.mark.parametrize("s_max", [0, 1, 40, 63, 64, 130])
def test_granulometry_sizes(s_max):
    check_granulometry(image((90, 130), np.uint8, seed=s_max), s_max, f"s_max={s_max}")


def test_granulometry_is_deterministic():
    F = dev(image((300, 411), np.float32, seed=2))
    a = gc.granulometry(F, 5)
    for _ in range(3):
        assert gc.granulometry(F, 5) == a


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("s_max", [0, 1, 3])
def test_asf_parity(dtype, shape, s_max):
    f = image(shape, dtype, seed=shape[1] + s_max)
    got = host(gc.asf(dev(f), s_max))
    assert np.array_equal(got, oracle.asf(f, s_max))


def test_asf_in_place():
    f = image((150, 260), np.float64, seed=9)
    F = dev(f)
    gc.asf(F, 3, out=F)
    assert np.array_equal(host(F), oracle.asf(f, 3))


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("shape", [(1, 1), (1, 300), (300, 1), (5, 7), (67, 129), (200, 517), (513, 385)])
@pytest.mark.parametrize("s_max", [2, 7])
def test_asf_mixed_chains(dtype, shape, s_max):
    """u8 and f32 ASF run their short chains as one chain with a dilation
    or an erosion per step, 32 steps per launch, so launches switch ops in
    their middle and the border fence changes sides (f64 runs each chain on
    its own); with the window path off, every chain of s_max = 7 (up to 14
    steps) goes that way."""
    f = image(shape, dtype, seed=7 * shape[0] + shape[1] + s_max)
    ref = oracle.asf(f, s_max)
    assert np.array_equal(host(gc.asf(dev(f), s_max)), ref)
    gc.set_window_path(-1)
    try:
        F = dev(f)
        gc.asf(F, s_max, out=F)   # in place as well
        assert np.array_equal(host(F), ref)
    finally:
        gc.set_window_path(0)


@pytest.mark.parametrize("dtype", [np.uint8, np.float32])
def test_asf_mixed_and_window_chains(dtype):
    """s_max = 20: the chains long enough for the window path (26 steps and
    more for u8, 34 for f32) take it, the shorter ones before and after them
    run as mixed chains."""
    f = image((300, 410), dtype, seed=16)
    assert np.array_equal(host(gc.asf(dev(f), 20)), oracle.asf(f, 20))


def test_full_size_u8_pattern_spectrum_and_asf():
    f = workloads.operator_u8()
    check_granulometry(f, 11, "1024x1024 PS[0,11]")
    assert np.array_equal(host(gc.asf(dev(f), 11)), oracle.asf(f, 11))
