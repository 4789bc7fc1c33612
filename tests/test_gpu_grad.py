"""GPU parity of the differentiable chain: per-step codes bit-exact against
the oracle's tie rule, the reverse gather against the oracle's scatter
(float64: same summation order; float32: 1e-5 relative), exact finite
differences on tie-free inputs, checkpointing invariance, and the
16 x 1024 x 1024 float32 200-step workload: every image's forward and
both gradients checked against the oracle."""
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


@pytest.mark.parametrize("op", OPS)
def test_autograd_exact_finite_differences(op):
    # Integer leaves, all distinct (no ties anywhere); eps = 1/4 and integer
    # upstream gradients keep every quantity exact in float64.
    shape, n = (6, 7), 5
    f, m = workloads.tie_free(*shape, seed=13)
    if op == "erode":
        f, m = m, f
    g = np.random.default_rng(2).integers(-4, 5, size=shape).astype(np.float64)
    F = dev(f).requires_grad_(True)
    M = dev(m).requires_grad_(True)
    y = gc.geodesic_chain(F, M, n, op=op, checkpoint_every=2)
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
        (gc.geodesic_chain(F, M, n, checkpoint_every=ck) * g).sum().backward()
        grads.append((host(F.grad), host(M.grad)))
    for a, b in grads[1:]:
        assert np.array_equal(a, grads[0][0]) and np.array_equal(b, grads[0][1])
    ref_gf, ref_gm = oracle.chain_vjp(oracle.DILATE, f, m, n, host(g))
    assert np.array_equal(grads[0][0], ref_gf) and np.array_equal(grads[0][1], ref_gm)


def test_batched_images_and_zero_steps():
    f, m = rand_pair((3, 40, 50), np.float32, seed=8)
    F = dev(f).requires_grad_(True)
    M = dev(m).requires_grad_(True)
    g = np.random.default_rng(1).standard_normal((3, 40, 50)).astype(np.float32)
    (gc.geodesic_chain(F, M, 17, op="erode", checkpoint_every=5) * dev(g)).sum().backward()
    for b in range(3):
        rf, rm = oracle.chain_vjp(oracle.ERODE, f[b], m[b], 17, g[b])
        np.testing.assert_allclose(host(F.grad)[b], rf, rtol=1e-5, atol=1e-5)
        np.testing.assert_allclose(host(M.grad)[b], rm, rtol=1e-5, atol=1e-5)
    F0 = dev(f).requires_grad_(True)
    M0 = dev(m).requires_grad_(True)
    (gc.geodesic_chain(F0, M0, 0) * dev(g)).sum().backward()
    assert np.array_equal(host(F0.grad), g) and not host(M0.grad).any()


@pytest.fixture(scope="module")
def differentiable_workload():
    """16 x 1024 x 1024 float32, 200 geodesic dilations, upstream N(0,1),
    checkpoint every 32 steps: inputs, forward result and both gradients,
    copied to the host."""
    f, m, g = workloads.differentiable_f32()
    F = dev(f).requires_grad_(True)
    M = dev(m).requires_grad_(True)
    y = gc.geodesic_chain(F, M, 200, op="dilate", checkpoint_every=32)
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
