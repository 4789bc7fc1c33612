"""GPU parity of gc_geodesic_chain_batch (a batch of equal-shape chains in
the same launches) against the oracle, image by image and bit-exact: every
dtype, dilation and erosion, ragged shapes over several tiles, strided and
pitched batches, in place, zero steps, one image, and the 16 x 1024 x 1024
float32 200-step forward of the differentiable workload (sampled images)."""
import numpy as np
import pytest
import torch

import oracle
import workloads
import paper_1911_13074_amd as gc

pytestmark = pytest.mark.gpu


def rand_batch(b, h, w, dtype, seed, levels=6):
    rng = np.random.default_rng(seed)
    if np.dtype(dtype) == np.uint8:
        f = (rng.integers(0, levels, size=(b, h, w)) * (255 // (levels - 1))).astype(np.uint8)
        m = (rng.integers(0, levels, size=(b, h, w)) * (255 // (levels - 1))).astype(np.uint8)
    else:
        f = rng.standard_normal((b, h, w)).astype(dtype)
        m = rng.standard_normal((b, h, w)).astype(dtype)
    return f, m


def code_of(op):
    return oracle.DILATE if op == "dilate" else oracle.ERODE


@pytest.mark.parametrize("dtype", [np.uint8, np.float32, np.float64])
@pytest.mark.parametrize("op", ["dilate", "erode"])
@pytest.mark.parametrize("b,h,w,n", [(1, 70, 90, 9), (3, 257, 190, 45), (5, 130, 400, 100), (2, 1, 300, 7)])
def test_batch_matches_oracle(dtype, op, b, h, w, n):
    f, m = rand_batch(b, h, w, dtype, seed=b * 1000 + h + w + n)
    out = gc.geodesic_chain_batch(op, torch.from_numpy(f).cuda(), torch.from_numpy(m).cuda(), n)
    got = out.cpu().numpy()
    for i in range(b):
        assert np.array_equal(got[i], oracle.chain(code_of(op), f[i], n, m[i])), f"image {i}"


def test_strided_pitched_in_place_and_zero_steps():
    """Images 300 elements apart inside a larger buffer, rows padded to a
    pitch of 120; in place (out = marker) with an odd number of launches;
    zero steps copies."""
    f, m = rand_batch(4, 90, 100, np.float32, seed=77)
    big_f = torch.full((4, 92, 120), -7.0, dtype=torch.float32, device="cuda")
    big_m = torch.full_like(big_f, -7.0)
    F, M = big_f[:, :90, :100], big_m[:, :90, :100]
    F.copy_(torch.from_numpy(f).cuda())
    M.copy_(torch.from_numpy(m).cuda())
    out = gc.geodesic_chain_batch("erode", F, M, 70, out=F)   # 3 launches of up to 32 steps
    got = out.cpu().numpy()
    for i in range(4):
        assert np.array_equal(got[i], oracle.chain(oracle.ERODE, f[i], 70, m[i])), f"image {i}"
    # padding untouched
    assert (big_f[:, 90:, :] == -7.0).all() and (big_f[:, :, 100:] == -7.0).all()
    z = gc.geodesic_chain_batch("dilate", torch.from_numpy(f).cuda(), torch.from_numpy(m).cuda(), 0)
    assert np.array_equal(z.cpu().numpy(), f)


def test_differentiable_workload_forward():
    """The 16 x 1024^2 f32 200-step forward the autograd function runs, in
    one batch call: images 0, 7 and 15 against the oracle."""
    f, m, _ = workloads.differentiable_f32()
    out = gc.geodesic_chain_batch("dilate", torch.from_numpy(f).cuda(), torch.from_numpy(m).cuda(), 200)
    got = out.cpu().numpy()
    for i in (0, 7, 15):
        assert np.array_equal(got[i], oracle.chain(oracle.DILATE, f[i], 200, m[i])), f"image {i}"
