"""GPU parity of the differentiable chain: per-step codes bit-exact against
the oracle's tie rule, the reverse gather against the oracle's scatter
(float64: same summation order; float32: 1e-5 relative), source ids
bit-exact against the ends of the oracle's code paths, the reverse pass
through them against the oracle's scatter (float64: 1e-12; float32: 1e-5),
exact finite differences on tie-free inputs for both methods, checkpointing
invariance, and the 16 x 1024 x 1024 float32 200-step workload: every
image's forward and both gradients checked against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import workloads
import paper_1911_13074_amd as gc

pytestmark = pytest.mark.gpu

OPS = ["dilate", "erode"]


def code_of(op):
    return oracle.DILATE if op == "dilate" else oracle.ERODE


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def rand_pair(shape, dtype, seed, levels=None):
    rng = np.random.default_rng(seed)
    if levels:
        f = rng.integers(0, levels, size=shape).astype(dtype)
        m = rng.integers(0, levels, size=shape).astype(dtype)
    else:
        f = rng.standard_normal(shape).astype(dtype)
        m = rng.standard_normal(shape).astype(dtype)
    return f, m


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("shape,levels", [((1, 1), None), ((1, 70), 3), ((33, 1), 3), ((37, 129), 4),
                                          ((70, 65), None), ((130, 200), 6)])
def test_codes_match_oracle(dtype, op, shape, levels):
    f, m = rand_pair(shape, dtype, seed=shape[0] + 3 * shape[1], levels=levels)
    n = 9
    out, codes = gc.geodesic_chain_fwd_codes(op, dev(f), dev(m), n)
    ref_out, ref_codes = oracle.chain_codes(code_of(op), f, n, m)
    assert np.array_equal(host(out), ref_out)
    assert np.array_equal(host(codes)[0], ref_codes)


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("levels", [None, 5])
def test_reverse_gather_float64_matches_scatter(op, levels):
    shape, n = (61, 97), 23
    f, m = rand_pair(shape, np.float64, seed=7, levels=levels)
    g = np.random.default_rng(3).standard_normal(shape)
    _, codes = gc.geodesic_chain_fwd_codes(op, dev(f), dev(m), n)
    gm = torch.zeros(shape, dtype=torch.float64, device="cuda")
    gf = gc.geodesic_chain_bwd(op, codes, dev(g), gm)
    ref_gf, ref_gm = oracle.chain_vjp(code_of(op), f, m, n, g)
    # same codes, same summation order, float64 on both sides
    assert np.array_equal(host(gf), ref_gf)
    assert np.array_equal(host(gm), ref_gm)


@pytest.mark.parametrize("op", OPS)
def test_reverse_gather_float32(op):
    shape, n = (128, 300), 40
    f, m = rand_pair(shape, np.float32, seed=11)
    g = np.random.default_rng(4).standard_normal(shape).astype(np.float32)
    _, codes = gc.geodesic_chain_fwd_codes(op, dev(f), dev(m), n)
    gm = torch.zeros(shape, dtype=torch.float32, device="cuda")
    gf = gc.geodesic_chain_bwd(op, codes, dev(g), gm)
    ref_gf, ref_gm = oracle.chain_vjp(code_of(op), f, m, n, g)
    for got, ref in ((host(gf), ref_gf), (host(gm), ref_gm)):
        np.testing.assert_allclose(got, ref, rtol=1e-5, atol=1e-5 * np.abs(ref).max())


@pytest.mark.parametrize("method", ["sources", "codes"])
@pytest.mark.parametrize("op", OPS)
def test_autograd_exact_finite_differences(op, method):
    # Integer leaves, all distinct (no ties anywhere); eps = 1/4 and integer
    # upstream gradients keep every quantity exact in float64.
    shape, n = (6, 7), 5
    f, m = workloads.tie_free(*shape, seed=13)
    if op == "erode":
        f, m = m, f
    g = np.random.default_rng(2).integers(-4, 5, size=shape).astype(np.float64)
    F = dev(f).requires_grad_(True)
    M = dev(m).requires_grad_(True)
    y = gc.geodesic_chain(F, M, n, op=op, checkpoint_every=2, method=method)
    (y * dev(g)).sum().backward()
    chain = gc.geodesic_dilate_chain if op == "dilate" else gc.geodesic_erode_chain

    def loss(ff, mm):
        return float((host(chain(dev(ff), dev(mm), n)) * g).sum())

    eps = 0.25
    for leaf, grad, is_marker in ((f, host(F.grad), True), (m, host(M.grad), False)):
        for idx in np.ndindex(*shape):
            p = leaf.copy(); p[idx] += eps
            q = leaf.copy(); q[idx] -= eps
            fd = ((loss(p, m) - loss(q, m)) if is_marker else (loss(f, p) - loss(f, q))) / (2 * eps)
            assert fd == grad[idx], (idx, fd, grad[idx])


def test_checkpointing_does_not_change_gradients():
    shape, n = (90, 110), 100
    f, m = rand_pair(shape, np.float64, seed=21)
    g = dev(np.random.default_rng(5).standard_normal(shape))
    grads = []
    for ck in (1, 7, 32, 1000):
        F = dev(f).requires_grad_(True)
        M = dev(m).requires_grad_(True)
        (gc.geodesic_chain(F, M, n, checkpoint_every=ck, method="codes") * g).sum().backward()
        grads.append((host(F.grad), host(M.grad)))
    for a, b in grads[1:]:
        assert np.array_equal(a, grads[0][0]) and np.array_equal(b, grads[0][1])
    ref_gf, ref_gm = oracle.chain_vjp(oracle.DILATE, f, m, n, host(g))
    assert np.array_equal(grads[0][0], ref_gf) and np.array_equal(grads[0][1], ref_gm)


@pytest.mark.parametrize("method", ["sources", "codes"])
def test_batched_images_and_zero_steps(method):
    f, m = rand_pair((3, 40, 50), np.float32, seed=8)
    F = dev(f).requires_grad_(True)
    M = dev(m).requires_grad_(True)
    g = np.random.default_rng(1).standard_normal((3, 40, 50)).astype(np.float32)
    (gc.geodesic_chain(F, M, 17, op="erode", checkpoint_every=5, method=method) * dev(g)).sum().backward()
    for b in range(3):
        rf, rm = oracle.chain_vjp(oracle.ERODE, f[b], m[b], 17, g[b])
        np.testing.assert_allclose(host(F.grad)[b], rf, rtol=1e-5, atol=1e-5)
        np.testing.assert_allclose(host(M.grad)[b], rm, rtol=1e-5, atol=1e-5)
    F0 = dev(f).requires_grad_(True)
    M0 = dev(m).requires_grad_(True)
    (gc.geodesic_chain(F0, M0, 0, method=method) * dev(g)).sum().backward()
    assert np.array_equal(host(F0.grad), g) and not host(M0.grad).any()


def test_sources_forward_without_gradients_and_mask_only():
    """With method='sources' a forward that no backward can follow (grad
    mode off, or inputs that need no gradient) runs the plain chain: the
    same output, bit-exact against the oracle; with only the mask
    requiring a gradient, the ids are kept and the mask gradient matches
    the oracle's."""
    f, m = rand_pair((2, 45, 70), np.float32, seed=12, levels=5)
    g = np.random.default_rng(3).standard_normal((2, 45, 70)).astype(np.float32)
    F = dev(f).requires_grad_(True)
    M = dev(m).requires_grad_(True)
    y = gc.geodesic_chain(F, M, 21)
    with torch.no_grad():
        y0 = gc.geodesic_chain(F, M, 21)
    y1 = gc.geodesic_chain(dev(f), dev(m), 21)
    assert y.requires_grad and not y0.requires_grad and not y1.requires_grad
    for b in range(2):
        ref = oracle.chain(oracle.DILATE, f[b], 21, m[b])
        for out in (y, y0, y1):
            assert np.array_equal(host(out)[b], ref), f"image {b}"
    M2 = dev(m).requires_grad_(True)
    (gc.geodesic_chain(dev(f), M2, 21) * dev(g)).sum().backward()
    for b in range(2):
        _, rm = oracle.chain_vjp(oracle.DILATE, f[b], m[b], 21, g[b])
        np.testing.assert_allclose(host(M2.grad)[b], rm, rtol=1e-5, atol=1e-5 * max(np.abs(rm).max(), 1))


@pytest.fixture(scope="module")
def differentiable_workload():
    """16 x 1024 x 1024 float32, 200 geodesic dilations, upstream N(0,1),
    checkpoint every 32 steps: inputs, forward result and both gradients,
    copied to the host."""
    f, m, g = workloads.differentiable_f32()
    F = dev(f).requires_grad_(True)
    M = dev(m).requires_grad_(True)
    y = gc.geodesic_chain(F, M, 200, op="dilate", checkpoint_every=32, method="sources")
    (y * dev(g)).sum().backward()
    res = (f, m, g, host(y), host(F.grad), host(M.grad))
    del F, M, y
    torch.cuda.empty_cache()
    return res


@pytest.mark.parametrize("chunk", range(4))
def test_differentiable_workload_full_size(differentiable_workload, chunk):
    """Every image of the differentiable workload (images b with b mod 4 ==
    chunk): the forward bit-exact against the oracle's chain, both
    gradients against the oracle's reference gradient (same tie rule) at
    1e-5 relative to the largest reference magnitude."""
    f, m, g, y, gf, gm = differentiable_workload
    assert y.shape == (16, 1024, 1024)
    for b in range(chunk, 16, 4):
        ref_y = oracle.chain(oracle.DILATE, f[b], 200, m[b])
        assert np.array_equal(y[b], ref_y), f"forward, image {b}"
        rf, rm = oracle.chain_vjp(oracle.DILATE, f[b], m[b], 200, g[b])
        np.testing.assert_allclose(gf[b], rf, rtol=1e-5, atol=1e-5 * np.abs(rf).max(), err_msg=f"marker {b}")
        np.testing.assert_allclose(gm[b], rm, rtol=1e-5, atol=1e-5 * np.abs(rm).max(), err_msg=f"mask {b}")


def test_differentiable_workload_gradient_mass(differentiable_workload):
    """Every unit of upstream gradient lands on a leaf: the two gradients
    sum to the upstream sum (float32 accumulation)."""
    _, _, g, _, gf, gm = differentiable_workload
    np.testing.assert_allclose(gf.astype(np.float64).sum() + gm.astype(np.float64).sum(),
                               g.astype(np.float64).sum(), rtol=1e-4)


# ---- source ids -------------------------------------------------------------
def sources_from_codes(codes):
    """Ends of the oracle's code paths: for every pixel of the final state,
    follow its code at the last step, then the code of the pixel it names at
    the step before, ..., to a pixel of the initial state or to a step where
    the mask won.  Returns int32 ids: y * X + x, with the top bit set for a
    mask pixel (the layout of a dense image)."""
    n, Y, X = codes.shape
    yy, xx = np.meshgrid(np.arange(Y), np.arange(X), indexing="ij")
    yy, xx = yy.ravel().copy(), xx.ravel().copy()
    at_mask = np.zeros(Y * X, dtype=bool)
    for t in range(n - 1, -1, -1):
        live = ~at_mask
        c = codes[t][yy[live], xx[live]].astype(np.int64)
        won = c == 9
        idx = np.flatnonzero(live)
        at_mask[idx[won]] = True
        moving = idx[~won]
        cm = c[~won]
        yy[moving] += cm // 3 - 1
        xx[moving] += cm % 3 - 1
    ids = (yy * X + xx).astype(np.uint32)
    ids[at_mask] |= np.uint32(0x80000000)
    return ids.view(np.int32).reshape(Y, X)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("shape,levels,n", [((1, 1), None, 3), ((1, 70), 3, 9), ((33, 1), 3, 17),
                                            ((37, 129), 4, 9), ((70, 65), None, 8), ((130, 200), 6, 25),
                                            ((61, 97), 2, 40), ((300, 260), 5, 21)])
def test_sources_match_oracle_paths(dtype, op, shape, levels, n):
    """Source ids are bit-exact against the ends of the oracle's code paths
    (one launch per 8 steps, so 9, 17, 25 and 40 steps chain the ids through
    several launches; 130 x 200 spans several cores with ragged ends, and
    300 x 260 has tiles whose whole region lies inside the image, which load
    without per-pixel tests; few levels give many ties)."""
    f, m = rand_pair(shape, dtype, seed=shape[0] * 7 + shape[1] + n, levels=levels)
    out, src = gc.geodesic_chain_fwd_sources(op, dev(f), dev(m), n)
    ref_out, ref_codes = oracle.chain_codes(code_of(op), f, n, m)
    assert np.array_equal(host(out), ref_out)
    assert np.array_equal(host(src), sources_from_codes(ref_codes))


@pytest.mark.parametrize("dtype,col0,rows,n", [(np.float64, 0, 50, 13), (np.float32, 0, 150, 21),
                                               (np.float32, 1, 150, 21)])
def test_sources_pitched_batch_and_zero_steps(dtype, col0, rows, n):
    """A batch of three pitched images (ids are offsets y * pitch + x within
    each image) and a zero-step chain (every pixel its own source), in
    float64 and in float32, the latter also as views that start at an odd
    column and span two rows of cores."""
    rng = np.random.default_rng(17)
    big_f = torch.zeros((3, rows, 80), dtype=getattr(torch, np.dtype(dtype).name), device="cuda")
    big_m = torch.zeros_like(big_f)
    f = rng.integers(0, 5, size=(3, rows, 70)).astype(dtype)
    m = rng.integers(0, 5, size=(3, rows, 70)).astype(dtype)
    F, M = big_f[:, :, col0:col0 + 70], big_m[:, :, col0:col0 + 70]
    F.copy_(dev(f))
    M.copy_(dev(m))
    out, src = gc.geodesic_chain_fwd_sources("dilate", F, M, n)
    s = host(src).view(np.uint32)
    for b in range(3):
        ref_out, codes = oracle.chain_codes(oracle.DILATE, f[b], n, m[b])
        assert np.array_equal(host(out)[b], ref_out), f"image {b}"
        ref = sources_from_codes(codes).view(np.uint32)
        pos = ref & 0x7FFFFFFF
        want = (pos // 70) * 80 + pos % 70 | (ref & 0x80000000)
        assert np.array_equal(s[b], want), f"image {b}"
    _, src0 = gc.geodesic_chain_fwd_sources("erode", dev(f[0]), dev(m[0]), 0)
    assert np.array_equal(host(src0), np.arange(rows * 70, dtype=np.int32).reshape(rows, 70))


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("dtype,levels", [(np.float64, None), (np.float64, 5), (np.float32, None), (np.float32, 4)])
def test_reverse_pass_through_sources(op, dtype, levels):
    """The scatter through source ids against the oracle's step-by-step
    scatter: the same contributions added in another order (float64 to
    1e-12, float32 to 1e-5 of the largest magnitude); the mask gradient is
    accumulated onto what grad_mask held."""
    shape, n = (96, 131), 37
    f, m = rand_pair(shape, dtype, seed=29, levels=levels)
    g = np.random.default_rng(6).standard_normal(shape).astype(dtype)
    _, src = gc.geodesic_chain_fwd_sources(op, dev(f), dev(m), n)
    prior = np.random.default_rng(7).standard_normal(shape).astype(dtype)
    gm = dev(prior.copy())
    gf = gc.geodesic_chain_bwd_sources(src, dev(g), gm)
    ref_gf, ref_gm = oracle.chain_vjp(code_of(op), f, m, n, g)
    tol = 1e-12 if dtype == np.float64 else 1e-5
    np.testing.assert_allclose(host(gf), ref_gf, rtol=tol, atol=tol * np.abs(ref_gf).max())
    np.testing.assert_allclose(host(gm) - prior, ref_gm, rtol=tol, atol=tol * max(np.abs(ref_gm).max(), 1))


@pytest.mark.parametrize("case", range(24))
def test_sources_random_configurations(case):
    """Seeded random sweep of the source-id path: dtype, op, shape (1 to 400
    per side, so one to several tiles, interior ones included), steps (1 to
    70, one to nine launches) and value levels; the forward bit-exact, the
    reverse pass against the oracle's scatter."""
    rng = np.random.default_rng(7000 + case)
    dtype = [np.float32, np.float64][int(rng.integers(0, 2))]
    op = OPS[int(rng.integers(0, 2))]
    h, w = int(rng.integers(1, 401)), int(rng.integers(1, 401))
    n = int(rng.choice([1, 2, int(rng.integers(3, 17)), int(rng.integers(17, 71))]))
    f, m = rand_pair((h, w), dtype, seed=case, levels=int(rng.choice([2, 6, 50])))
    g = rng.standard_normal((h, w)).astype(dtype)
    what = f"case {case}: {np.dtype(dtype)} {op} {h}x{w} n={n}"
    out, src = gc.geodesic_chain_fwd_sources(op, dev(f), dev(m), n)
    ref_out, _ = oracle.chain_codes(code_of(op), f, n, m)
    assert np.array_equal(host(out), ref_out), what
    gm = torch.zeros((h, w), dtype=out.dtype, device="cuda")
    gf = gc.geodesic_chain_bwd_sources(src, dev(g), gm)
    rgf, rgm = oracle.chain_vjp(code_of(op), f, m, n, g)
    tol = 1e-12 if dtype == np.float64 else 1e-5
    np.testing.assert_allclose(host(gf), rgf, rtol=tol, atol=tol * max(np.abs(rgf).max(), 1), err_msg=what)
    np.testing.assert_allclose(host(gm), rgm, rtol=tol, atol=tol * max(np.abs(rgm).max(), 1), err_msg=what)


def test_methods_agree_on_checkpointing():
    """Both methods, several checkpoint spacings, one float64 chain: the
    gradients agree with the oracle's to 1e-12."""
    shape, n = (90, 110), 100
    f, m = rand_pair(shape, np.float64, seed=21, levels=7)
    g = dev(np.random.default_rng(5).standard_normal(shape))
    ref_gf, ref_gm = oracle.chain_vjp(oracle.DILATE, f, m, n, host(g))
    for method in ("sources", "codes"):
        for ck in (1, 9, 32, 1000):
            F = dev(f).requires_grad_(True)
            M = dev(m).requires_grad_(True)
            (gc.geodesic_chain(F, M, n, checkpoint_every=ck, method=method) * g).sum().backward()
            np.testing.assert_allclose(host(F.grad), ref_gf, rtol=1e-12, atol=1e-12 * np.abs(ref_gf).max())
            np.testing.assert_allclose(host(M.grad), ref_gm, rtol=1e-12, atol=1e-12 * np.abs(ref_gm).max())


def test_reverse_pass_ignores_ids_beyond_the_image():
    """Ids whose offset lies beyond the image are skipped: a source map with
    some ids overwritten by such values gives the gradient of the valid ids
    alone (and nothing is written outside the gradient images)."""
    shape, n = (40, 50), 12
    f, m = rand_pair(shape, np.float32, seed=31)
    _, src = gc.geodesic_chain_fwd_sources("dilate", dev(f), dev(m), n)
    bad = src.clone()
    rng = np.random.default_rng(9)
    ys, xs = rng.integers(0, 40, size=30), rng.integers(0, 50, size=30)
    vals = [0x7FFFFFFF, 40 * 50, 40 * 50 + 123, -1]   # -1: the mask bit and offset 2^31 - 1
    for i, (y, x) in enumerate(zip(ys, xs)):
        bad[y, x] = int(np.int32(np.uint32(vals[i % 4]) if vals[i % 4] >= 0 else -1))
    g = np.random.default_rng(10).standard_normal(shape).astype(np.float32)
    guard = torch.full((3, 40, 50), 5.0, dtype=torch.float32, device="cuda")
    gf, gm = guard[0], guard[1]
    gm.zero_()
    gc.geodesic_chain_bwd_sources(bad, dev(g), gm, grad_marker=gf)
    # the reference: drop the contributions of the overwritten pixels
    g_valid = g.copy()
    g_valid[ys, xs] = 0
    gf_ref = torch.zeros(shape, dtype=torch.float32, device="cuda")
    gm_ref = torch.zeros(shape, dtype=torch.float32, device="cuda")
    gc.geodesic_chain_bwd_sources(src, dev(g_valid), gm_ref, grad_marker=gf_ref)
    np.testing.assert_allclose(host(gf), host(gf_ref), rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(host(gm), host(gm_ref), rtol=1e-6, atol=1e-6)
    assert (host(guard[2]) == 5.0).all()
