"""The HIP-error path, forced from the host: with GEOCHAIN_INJECT_HIP_FAULT
set, a checked HIP call whose text contains the given name is not made and
the entry point returns GC_ERR_HIP with a detail message.  Each case runs in
a child process, since the library reads the variable once."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_child(code, inject, extra_env=None):
    env = dict(os.environ)
    env["GEOCHAIN_INJECT_HIP_FAULT"] = inject
    env.update(extra_env or {})
    r = subprocess.run([sys.executable, "-c", textwrap.dedent(code)], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    return r.stdout


CPU_CASE = """
    import ctypes, sys
    sys.path.insert(0, ".")
    from paper_1911_13074_amd import abi
    FAKE = 1 << 40
    s = abi.gc_shape(64, 64, 64)
    st = abi.gc_geodesic_dilate_chain(abi.GC_U8, FAKE, FAKE + (1 << 20), FAKE + (2 << 20), s, 40, None)
    assert st == abi.GC_ERR_HIP, st
    msg = abi.last_error()
    assert "hipGetDevice" in msg and "injected fault" in msg, msg
    steps = ctypes.c_int64(5)
    st = abi.gc_reconstruct_by_erosion(abi.GC_F32, FAKE, FAKE + (1 << 20), FAKE + (2 << 20), s, -1,
                                       ctypes.byref(steps), None)
    assert st == abi.GC_ERR_HIP and "injected fault" in abi.last_error() and steps.value == 0
    # validation still answers first: no HIP call is reached
    assert abi.gc_dilate_chain(abi.GC_U8, FAKE, FAKE + 8, s, 3, None) == abi.GC_ERR_ALIAS
    print("ok")
"""


def test_injected_fault_reaches_the_caller():
    assert run_child(CPU_CASE, "hipGetDevice").strip().endswith("ok")


GPU_CASE = """
    import sys
    sys.path.insert(0, ".")
    import numpy as np, torch
    import oracle, workloads
    import paper_1911_13074_amd as gc
    from paper_1911_13074_amd import abi
    f, m = workloads.small_u8()
    F, M = torch.from_numpy(f).cuda(), torch.from_numpy(m).cuda()
    print("case: n = 0 copies through hipMemcpy2DAsync, which is made to fail", flush=True)
    try:
        gc.geodesic_dilate_chain(F, M, 0)
        raise SystemExit("no error")
    except gc.GeochainError as e:
        assert e.status == abi.GC_ERR_HIP and "injected fault" in str(e), str(e)
    print("case: a chain that makes no copy still runs and is exact", flush=True)
    out = gc.geodesic_dilate_chain(F, M, 50)
    assert np.array_equal(out.cpu().numpy(), oracle.chain(oracle.DILATE, f, 50, m))
    print("ok", flush=True)
"""


@pytest.mark.gpu
def test_injected_fault_on_gpu_leaves_library_usable():
    assert run_child(GPU_CASE, "hipMemcpy2DAsync").strip().endswith("ok")
