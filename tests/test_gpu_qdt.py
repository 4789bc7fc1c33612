"""GPU parity of the quasi-distance transform (Eq. 13-15) through the C ABI
against the oracle: the distance d and d_L1 (int32) and the residual are
bit-exact (min, one subtraction and integer increments), and the erosion and
eta step counts are equal; on ragged shapes across many tiles, both tile
layouts (one and two columns per lane), padded pitches, the constructed
case where eta lowers a jump of six, and the 1024 x 1024 u8 image."""
import numpy as np
import pytest
import torch

import oracle
import workloads
import paper_1911_13074_amd as gc
from paper_1911_13074_amd import abi

pytestmark = pytest.mark.gpu

DTYPES = [np.uint8, np.float32, np.float64]
SHAPES = [(1, 1), (1, 300), (300, 1), (2, 3), (67, 129), (200, 517), (513, 385)]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def assert_same(got, expect, what):
    assert got.dtype == expect.dtype, what
    if not np.array_equal(got, expect):
        bad = np.argwhere(got != expect)
        y, x = bad[0]
        raise AssertionError(f"{what}: {len(bad)} pixels differ, first at (y={y}, x={x}): "
                             f"got {got[y, x]!r} expected {expect[y, x]!r}")


def image(shape, dtype, seed, kind):
    if kind == "levels":
        v = np.random.default_rng(seed).integers(0, 6, size=shape)
        return (v * 40).astype(dtype) if dtype == np.uint8 else (v * 0.3 - 0.7).astype(dtype)
    f = workloads.blur(shape[0], shape[1], 2.0, seed) if min(shape) > 1 else \
        np.random.default_rng(seed).integers(0, 256, size=shape).astype(np.uint8)
    return f if dtype == np.uint8 else (f / 255.0 * 2.0 - 0.5).astype(dtype)


def check(f, what):
    dl1, d, r, steps, eta = oracle.quasi_distance(f)
    F = dev(f)
    g_dl1, g_r, g_steps, g_eta = gc.quasi_distance(F, lipschitz=True, with_residual=True)
    assert (g_steps, g_eta) == (steps, eta), (what, g_steps, steps, g_eta, eta)
    assert_same(host(g_dl1), dl1, f"{what} d_L1")
    assert_same(host(g_r), r, f"{what} residual")
    g_d, none, g_steps2, g_eta2 = gc.quasi_distance(F, lipschitz=False)
    assert none is None and g_steps2 == steps and g_eta2 == 0
    assert_same(host(g_d), d, f"{what} d")


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("kind", ["levels", "smooth"])
def test_qdt_parity(dtype, shape, kind):
    check(image(shape, dtype, seed=shape[0] * 7 + shape[1], kind=kind), f"{kind} {shape}")


def test_eta_lowers_a_jump():
    row = np.array([0, 100, 100, 100, 100, 50, 100, 100, 75, 100, 100, 100], np.uint8)
    for reps in (3, 150):
        check(np.repeat(row[None, :], reps, axis=0), f"jump x{reps}")
        check(np.repeat(row[None, :], reps, axis=0).T.copy(), f"jump^T x{reps}")


@pytest.mark.parametrize("dtype", DTYPES)
def test_qdt_padded_pitch(dtype):
    h, w = 140, 203
    f = image((h, w), dtype, seed=4, kind="smooth")
    F = torch.zeros((h, 256), dtype=dev(f).dtype, device="cuda")
    F[:, :w] = dev(f)
    fv = F[:, :w]
    g_dl1, g_r, steps, eta = gc.quasi_distance(fv, with_residual=True)
    assert g_dl1.stride(0) == 256
    dl1, _, r, ref_steps, ref_eta = oracle.quasi_distance(f)
    assert (steps, eta) == (ref_steps, ref_eta)
    assert_same(host(g_dl1), dl1, "d_L1")
    assert_same(host(g_r), r, "residual")


def test_qdt_constant_and_empty():
    dl1, r, steps, eta = gc.quasi_distance(dev(np.full((50, 70), 9, np.uint8)), with_residual=True)
    assert steps == 0 and eta == 0 and not host(dl1).any() and not host(r).any()
    e = torch.empty((0, 5), dtype=torch.float32, device="cuda")
    dl1, _, steps, eta = gc.quasi_distance(e)
    assert dl1.shape == (0, 5) and steps == 0 and eta == 0


def test_qdt_full_size_u8():
    f = workloads.operator_u8()
    check(f, "1024x1024 u8")
