"""The geodesic chain entry point that allocates nothing
(gc_geodesic_chain_noalloc), called through the C ABI, against the chain
entry points that use the library's workspaces (gc_geodesic_dilate_chain /
gc_geodesic_erode_chain): bit-exact, since both only select existing values.

Calls follow one another on one device, each time through the same fixed
array: a large image and then a smaller one (the second call must not see
the first one's contents), u8 / f32 / f64, dilation and erosion, in place,
an odd number of launches, the largest image the array holds, and a fresh
stream, on which the call must not allocate.
"""
import ctypes

import numpy as np
import pytest
import torch

import workloads
from paper_1911_13074_amd import abi

pytestmark = pytest.mark.gpu

CODES = {torch.uint8: abi.GC_U8, torch.float32: abi.GC_F32, torch.float64: abi.GC_F64}


def shape_of(t):
    return abi.gc_shape(t.shape[1], t.shape[0], t.stride(0))


def stream_of(t):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def noalloc(op, marker, mask, out, n):
    st = abi.gc_geodesic_chain_noalloc(CODES[marker.dtype], op, marker.data_ptr(), mask.data_ptr(),
                                       out.data_ptr(), shape_of(marker), n, stream_of(marker))
    assert st == abi.GC_OK, abi.last_error()
    return out


def workspace_chain(op, marker, mask, n):
    out = torch.empty_like(marker)
    fn = abi.gc_geodesic_dilate_chain if op == abi.GC_DILATE else abi.gc_geodesic_erode_chain
    st = fn(CODES[marker.dtype], marker.data_ptr(), mask.data_ptr(), out.data_ptr(), shape_of(marker), n,
            stream_of(marker))
    assert st == abi.GC_OK, abi.last_error()
    return out


def inputs(h, w, dtype, op, seed):
    """Blurred-noise mask with the marker below it (dilation) or above it
    (erosion), as the chain workloads are built."""
    m = workloads.blur(h, w, 4.0, seed)
    if op == abi.GC_DILATE:
        f = np.maximum(m.astype(np.int16) - 40, 0).astype(np.uint8)
    else:
        f = np.minimum(m.astype(np.int16) + 40, 255).astype(np.uint8)
    if dtype != torch.uint8:
        rng = np.random.default_rng(seed + 1)
        jitter = rng.random((h, w))
        m = m.astype(np.float64) + jitter
        f = f.astype(np.float64) + jitter
    tf = torch.from_numpy(np.ascontiguousarray(f)).to("cuda", dtype)
    tm = torch.from_numpy(np.ascontiguousarray(m)).to("cuda", dtype)
    return tf, tm


def assert_equal(got, expect, what):
    torch.cuda.synchronize()
    g, e = got.cpu(), expect.cpu()
    if not torch.equal(g, e):
        bad = (g != e).nonzero()
        raise AssertionError(f"{what}: {bad.shape[0]} pixels differ, first at {tuple(bad[0].tolist())}")


@pytest.mark.parametrize("dtype", [torch.uint8, torch.float32, torch.float64])
@pytest.mark.parametrize("op", [abi.GC_DILATE, abi.GC_ERODE])
def test_two_calls_second_smaller(dtype, op):
    # 1024 x 1024 over 47 launches of up to 32 steps, then a ragged 300 x 517
    # image whose chain ends in a different buffer parity
    for (h, w, n, seed) in [(1024, 1024, 1500, 11), (300, 517, 77, 12)]:
        print(f"noalloc: {dtype} op={op} {h}x{w} n={n}", flush=True)
        f, m = inputs(h, w, dtype, op, seed)
        expect = workspace_chain(op, f, m, n)
        out = torch.empty_like(f)
        noalloc(op, f, m, out, n)
        assert_equal(out, expect, f"{h}x{w} n={n}")


def test_in_place_and_pitched():
    """In place (out = marker) with an odd number of launches, and a padded
    row pitch, each after a larger call."""
    f, m = inputs(512, 512, torch.uint8, abi.GC_DILATE, 21)
    expect = workspace_chain(abi.GC_DILATE, f, m, 96)
    noalloc(abi.GC_DILATE, f, m, torch.empty_like(f), 96)
    inplace = f.clone()
    noalloc(abi.GC_DILATE, inplace, m, inplace, 96)   # 3 launches of 32 steps
    assert_equal(inplace, expect, "in place, 96 steps")

    big_f = torch.zeros((200, 160), dtype=torch.float32, device="cuda")
    big_m = torch.zeros_like(big_f)
    f2, m2 = inputs(200, 150, torch.float32, abi.GC_ERODE, 22)
    pf, pm = big_f[:, :150], big_m[:, :150]
    pf.copy_(f2)
    pm.copy_(m2)
    expect = workspace_chain(abi.GC_ERODE, f2, m2, 41)
    out = torch.full((200, 160), -1.0, dtype=torch.float32, device="cuda")[:, :150]
    noalloc(abi.GC_ERODE, pf, pm, out, 41)
    assert_equal(out, expect, "pitched f32, 41 steps")


def test_largest_image_on_a_fresh_stream():
    """A 4096 x 4096 u8 image fills the 16 MiB array exactly; on a stream the
    library has never seen, the call leaves the device's free memory as it
    was (the workspace entry points would allocate 16 MiB for it)."""
    f, m = inputs(4096, 4096, torch.uint8, abi.GC_DILATE, 31)
    out = torch.empty_like(f)
    expect = workspace_chain(abi.GC_DILATE, f, m, 70)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        free_before = torch.cuda.mem_get_info()[0]
        noalloc(abi.GC_DILATE, f, m, out, 70)
        s.synchronize()
        free_after = torch.cuda.mem_get_info()[0]
    assert free_before - free_after < (16 << 20), (free_before, free_after)
    assert_equal(out, expect, "4096 x 4096, 70 steps")
    # and a small call after it on the default stream
    f3, m3 = inputs(64, 64, torch.uint8, abi.GC_DILATE, 32)
    out3 = torch.empty_like(f3)
    noalloc(abi.GC_DILATE, f3, m3, out3, 200)
    assert_equal(out3, workspace_chain(abi.GC_DILATE, f3, m3, 200), "64 x 64 after the largest")
