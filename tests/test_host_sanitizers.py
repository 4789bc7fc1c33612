"""The host layer under AddressSanitizer and UndefinedBehaviorSanitizer.

The library is built once more with the sanitizers on its host code only
(device code is built as usual, without them), and the host-side tests --
argument validation of every entry point, the torch wrappers' layout
checks and the injected HIP-error path -- run against that build in a
child process with the sanitizer runtime preloaded.  Any sanitizer report
fails the test.  No GPU is used: every call ends in validation or in a
failed (or injected) HIP call.  The build is cached in the system temp
directory, keyed by the sources."""
import hashlib
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1911_13074_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ASAN_RT = "/opt/rocm/llvm/lib/clang/22/lib/linux/libclang_rt.asan-x86_64.so"
HOST_TESTS = ["tests/test_abi.py", "tests/test_ops_validation.py", "tests/test_fault_injection.py",
              "tests/test_tune_cache.py"]


def sources_key():
    h = hashlib.sha256()
    for d in (CSRC, INCLUDE):
        for fn in sorted(os.listdir(d)):
            h.update(fn.encode())
            h.update(open(os.path.join(d, fn), "rb").read())
    return h.hexdigest()[:16]


@pytest.fixture(scope="module")
def sanitized_library():
    if not os.path.exists(HIPCC) or not os.path.exists(ASAN_RT):
        pytest.skip("hipcc or the clang ASan runtime is not installed")
    out_dir = os.path.join(tempfile.gettempdir(), f"geochain_hostsan_{sources_key()}")
    lib = os.path.join(out_dir, "libgeochain_hostsan.so")
    if not os.path.exists(lib):
        os.makedirs(out_dir, exist_ok=True)
        cmd = [HIPCC, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
               "-Xarch_device", "-fno-honor-nans", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
               "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
               "-I", INCLUDE, "-I", CSRC, "-o", lib + ".tmp", os.path.join(CSRC, "geochain.hip")]
        subprocess.run(cmd, check=True, capture_output=True, timeout=900)
        os.replace(lib + ".tmp", lib)
    return lib


def test_host_checks_clean_under_asan_and_ubsan(sanitized_library):
    env = dict(os.environ)
    env.update({
        "GEOCHAIN_LIB": sanitized_library,
        "LD_PRELOAD": ASAN_RT,
        "ASAN_OPTIONS": "detect_leaks=0:verify_asan_link_order=0:abort_on_error=1",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
    })
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider"]
                       + HOST_TESTS, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    report = r.stdout + r.stderr
    assert "AddressSanitizer" not in report and "runtime error:" not in report, report[-4000:]
    assert r.returncode == 0, report[-4000:]
    assert " passed" in r.stdout
