"""GPU parity of the large-window path for plain chains (one separable
(2n+1)^2 window by the van Herk / Gil-Werman scheme) against the oracle's
chain of n 3x3 steps, bit-exact for every dtype: ragged shapes, radii below,
at and beyond the image size, chunk and block boundaries, padded pitches, in
place, lines too long for the path (which then run as chains), and the
1024 x 1024 workloads; plus equality with the register-blocked chain."""
import numpy as np
import pytest
import torch

import oracle
import workloads
import paper_1911_13074_amd as gc

pytestmark = pytest.mark.gpu

DTYPES = [np.uint8, np.float32, np.float64]
OPS = [oracle.DILATE, oracle.ERODE]


@pytest.fixture(autouse=True)
def _window_always():
    gc.set_window_path(1)
    yield
    gc.set_window_path(0)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rand(shape, dtype, seed):
    rng = np.random.default_rng(seed)
    if np.dtype(dtype) == np.uint8:
        return rng.integers(0, 256, size=shape).astype(np.uint8)
    return rng.standard_normal(shape).astype(dtype)


def run(op, x, n, **kw):
    fn = gc.dilate_chain if op == oracle.DILATE else gc.erode_chain
    return fn(x, n, **kw)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("shape", [(1, 1), (1, 300), (300, 1), (2, 2), (67, 129), (200, 517), (64, 64)])
def test_window_parity(dtype, op, shape):
    for n in (1, 2, 15, 16, 31, 32, 33, 63, 64, 65, 100, 700):
        f = rand(shape, dtype, seed=n + shape[0])
        ref = oracle.chain(op, f, min(n, max(shape)), None)
        assert np.array_equal(host(run(op, dev(f), n)), ref), (n, shape)


@pytest.mark.parametrize("dtype", DTYPES)
def test_window_equals_chain_full_size(dtype):
    x = dev(workloads.plain_input(dtype))
    for n in (13, 24, 91, 183):
        for op in OPS:
            win = host(run(op, x, n))
            gc.set_window_path(-1)
            chain = host(run(op, x, n))
            gc.set_window_path(1)
            assert np.array_equal(win, chain), (n, op)


@pytest.mark.parametrize("dtype", DTYPES)
def test_window_padded_pitch_and_in_place(dtype):
    h, w = 150, 203
    f = rand((h, w), dtype, seed=1)
    F = torch.zeros((h, 256), dtype=dev(f).dtype, device="cuda")
    F[:, :w] = dev(f)
    fv = F[:, :w]
    out = run(oracle.ERODE, fv, 37)
    assert out.stride(0) == 256
    assert np.array_equal(host(out), oracle.chain(oracle.ERODE, f, 37))
    run(oracle.DILATE, fv, 29, out=fv)
    assert np.array_equal(host(fv), oracle.chain(oracle.DILATE, f, 29))
    assert torch.all(F[:, w:] == 0)


@pytest.mark.parametrize("dtype", [np.uint8, np.float32])
def test_long_lines_take_the_segment_loop_kernel(dtype):
    # 5000 + 2 * 50 padded pixels need 81 positions per lane: beyond the
    # register variants (up to 65), within the loop kernel's LDS buffer
    f = rand((3, 5000), dtype, seed=4)
    for op in OPS:
        assert np.array_equal(host(run(op, dev(f), 50)), oracle.chain(op, f, 50))
    g = rand((4800, 5), dtype, seed=5)
    assert np.array_equal(host(run(oracle.DILATE, dev(g), 60)), oracle.chain(oracle.DILATE, g, 60))


def test_lines_too_long_for_the_window_path_run_as_chains():
    # 30000 pixels per line exceed the path's LDS line buffer
    f = rand((3, 30000), np.uint8, seed=2)
    assert np.array_equal(host(run(oracle.DILATE, dev(f), 40)), oracle.chain(oracle.DILATE, f, 40))
    g = rand((30000, 2), np.float32, seed=3)
    assert np.array_equal(host(run(oracle.ERODE, dev(g), 30)), oracle.chain(oracle.ERODE, g, 30))


def test_operators_through_the_window_path():
    f = workloads.operator_u8(size=300)
    for s in (3, 30):
        out, steps, _ = gc.open_by_reconstruction(dev(f), s)
        ref, ref_steps, _ = oracle.open_by_reconstruction(f, s)
        assert steps == ref_steps and np.array_equal(host(out), ref)
    assert np.array_equal(host(gc.asf(dev(f), 4)), oracle.asf(f, 4))
    G, _ = gc.granulometry(dev(f), 6)
    assert G == list(oracle.granulometry(f, 6)[0])
