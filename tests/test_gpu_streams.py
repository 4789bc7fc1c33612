"""Concurrent calls: each (device, stream) pair has its own workspace, so
chains, reconstructions and plain chains issued at the same time from
several host threads, each on its own stream, give exactly what the same
calls give one after another on the default stream (which the oracle
checks for the first input).  Chains also record into a HIP graph once a
first call on the capturing stream has sized its workspace."""
import threading

import numpy as np
import pytest
import torch

import oracle
import paper_1911_13074_amd as gc

pytestmark = pytest.mark.gpu


def inputs(seed, shape):
    rng = np.random.default_rng(seed)
    f = rng.integers(0, 200, size=shape).astype(np.uint8)
    m = rng.integers(50, 256, size=shape).astype(np.uint8)
    return f, m


def work(F, M):
    a = gc.geodesic_dilate_chain(F, M, 77)
    r, steps, conv = gc.reconstruct_by_dilation(F, M)
    e = gc.erode_chain(F, 40)
    return a, r, steps, conv, e


def test_calls_from_threads_on_their_own_streams():
    shapes = [(300, 457), (129, 1030), (700, 64), (513, 513)]
    host_in = [inputs(10 + i, s) for i, s in enumerate(shapes)]
    cases = [(torch.from_numpy(f).cuda(), torch.from_numpy(m).cuda()) for f, m in host_in]
    ref = [work(F, M) for F, M in cases]
    torch.cuda.synchronize()
    f0, m0 = host_in[0]
    assert np.array_equal(ref[0][0].cpu().numpy(), oracle.chain(oracle.DILATE, f0, 77, m0))
    rref, rsteps, _ = oracle.reconstruct(oracle.DILATE, f0, m0)
    assert ref[0][2] == rsteps and np.array_equal(ref[0][1].cpu().numpy(), rref)
    assert np.array_equal(ref[0][4].cpu().numpy(), oracle.chain(oracle.ERODE, f0, 40))

    streams = [torch.cuda.Stream() for _ in cases]
    got = [None] * len(cases)
    errors = []

    def run(i):
        try:
            with torch.cuda.stream(streams[i]):
                outs = [work(*cases[i]) for _ in range(3)]
            streams[i].synchronize()
            got[i] = outs
        except Exception as ex:  # reported below, in the main thread
            errors.append((i, repr(ex)))

    threads = [threading.Thread(target=run, args=(i,)) for i in range(len(cases))]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=60)
    assert not any(t.is_alive() for t in threads)
    assert not errors, errors
    for i, outs in enumerate(got):
        a0, r0, s0, c0, e0 = ref[i]
        for a, r, s, c, e in outs:
            assert torch.equal(a, a0) and torch.equal(e, e0), i
            assert c and c0 and s == s0 and torch.equal(r, r0), i


def test_chains_captured_in_a_graph_replay_exactly():
    """Geodesic and plain chains (several launches each, ping-pong through
    the stream's workspace) captured after a warm-up call on the capturing
    stream; every replay, with eager library work and synchronisation
    between replays, equals the eager result, which the oracle checks."""
    f, m = inputs(41, (517, 389))
    F, M = torch.from_numpy(f).cuda(), torch.from_numpy(m).cuda()
    out_g = torch.empty_like(F)
    out_p = torch.empty_like(F)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        gc.geodesic_dilate_chain(F, M, 100, out=out_g)
        gc.erode_chain(F, 9, out=out_p)
    s.synchronize()
    ref_g, ref_p = out_g.clone(), out_p.clone()
    assert np.array_equal(ref_g.cpu().numpy(), oracle.chain(oracle.DILATE, f, 100, m))
    assert np.array_equal(ref_p.cpu().numpy(), oracle.chain(oracle.ERODE, f, 9))
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        gc.geodesic_dilate_chain(F, M, 100, out=out_g)
        gc.erode_chain(F, 9, out=out_p)
    for _ in range(4):
        out_g.zero_()
        out_p.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out_g, ref_g) and torch.equal(out_p, ref_p)
        gc.geodesic_erode_chain(F, M, 33)   # eager work on the default stream
        torch.cuda.synchronize()
