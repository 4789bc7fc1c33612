"""The C-ABI library loads and exports what include/geochain.h declares, and
its host-side argument checks answer before any GPU work (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_1911_13074_amd import abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"\b(gc_\w+)\s*\(", text)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = abi.load()
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name


def test_binding_covers_every_declared_symbol():
    assert set(declared_functions()) == set(abi.SIGNATURES)


def test_status_strings():
    assert abi.status_string(0) == "GC_OK"
    assert abi.status_string(-3) == "GC_ERR_ALIAS"
    assert abi.status_string(-6) == "GC_ERR_NOT_CONVERGED"
    assert abi.status_string(-99) == "GC_ERR_UNKNOWN"
    assert abi.gc_version() >= 100


def shape(w, h, p):
    return abi.gc_shape(w, h, p)


FAKE = 1 << 40  # never dereferenced: every call below fails validation first


@pytest.mark.parametrize("call", [
    # pitch < width
    lambda: abi.gc_geodesic_dilate_chain(abi.GC_U8, FAKE, FAKE + (1 << 20), FAKE + (2 << 20),
                                         shape(10, 10, 9), 3, None),
    # negative size
    lambda: abi.gc_dilate_chain(abi.GC_F32, FAKE, FAKE + (1 << 20), shape(-1, 10, 10), 3, None),
    # unknown dtype
    lambda: abi.gc_erode_chain(7, FAKE, FAKE + (1 << 20), shape(4, 4, 4), 1, None),
    # negative steps
    lambda: abi.gc_geodesic_erode_chain(abi.GC_F64, FAKE, FAKE + (1 << 20), FAKE + (2 << 20),
                                        shape(4, 4, 4), -2, None),
    # null pointers on a non-empty image
    lambda: abi.gc_geodesic_dilate_chain(abi.GC_U8, None, FAKE, FAKE + (1 << 20),
                                         shape(4, 4, 4), 1, None),
    lambda: abi.gc_geodesic_dilate_chain(abi.GC_U8, FAKE, None, FAKE + (1 << 20),
                                         shape(4, 4, 4), 1, None),
])
def test_invalid_arguments(call):
    assert call() == abi.GC_ERR_INVALID_ARG
    assert abi.last_error() != ""


def test_size_limits():
    """Sides above 2^25 and images above 2^36 pixels are refused before any
    HIP call (launch grids and tile counts stay within 32 bits)."""
    steps = ctypes.c_int64()
    for s in (shape((1 << 25) + 1, 1, (1 << 25) + 1), shape(1, (1 << 25) + 1, 1),
              shape(1 << 20, (1 << 16) + 1, 1 << 20)):
        far = 1 << 46
        assert abi.gc_geodesic_dilate_chain(abi.GC_U8, FAKE, FAKE + far, FAKE + 2 * far, s, 3,
                                            None) == abi.GC_ERR_UNSUPPORTED
        assert abi.gc_erode_chain(abi.GC_F32, FAKE, FAKE + far, s, 3, None) == abi.GC_ERR_UNSUPPORTED
        assert abi.gc_reconstruct_by_dilation(abi.GC_U8, FAKE, FAKE + far, FAKE + 2 * far, s, -1,
                                              ctypes.byref(steps), None) == abi.GC_ERR_UNSUPPORTED
        assert "not supported" in abi.last_error()


def test_plan_steps_validates():
    steps = (ctypes.c_int64 * 1)()
    assert abi.gc_plan_steps(None, steps) == abi.GC_ERR_INVALID_ARG


def test_aliasing_is_rejected():
    s = shape(100, 100, 128)
    # out == mask
    assert abi.gc_geodesic_dilate_chain(abi.GC_U8, FAKE, FAKE + (1 << 20), FAKE + (1 << 20),
                                        s, 5, None) == abi.GC_ERR_ALIAS
    # out overlaps the mask's last row
    assert abi.gc_geodesic_erode_chain(abi.GC_F32, FAKE, FAKE + (1 << 20),
                                       FAKE + (1 << 20) + 4 * 99 * 128, s, 5,
                                       None) == abi.GC_ERR_ALIAS
    # out partially overlaps the input of a plain chain
    assert abi.gc_dilate_chain(abi.GC_F64, FAKE, FAKE + 8, s, 5, None) == abi.GC_ERR_ALIAS
    steps = ctypes.c_int64(7)
    assert abi.gc_reconstruct_by_dilation(abi.GC_U8, FAKE, FAKE + (1 << 20), FAKE + (1 << 20), s,
                                          -1, ctypes.byref(steps), None) == abi.GC_ERR_ALIAS


def test_tuning_hook_validates():
    assert abi.gc_set_tuning(64, -1) == abi.GC_ERR_INVALID_ARG
    assert abi.gc_set_tuning(4, 9) == abi.GC_ERR_INVALID_ARG
    assert abi.gc_set_tuning(0, -1) == abi.GC_OK


def _steps():
    return ctypes.c_int64(123)


@pytest.mark.parametrize("call", [
    # h negative, NaN or infinite; u8 h not an integer
    lambda s: abi.gc_hmax(abi.GC_F32, FAKE, FAKE + (1 << 20), shape(8, 8, 8), -1.0, -1, s, None),
    lambda s: abi.gc_dome(abi.GC_F64, FAKE, FAKE + (1 << 20), shape(8, 8, 8), float("nan"), -1, s,
                          None),
    lambda s: abi.gc_hmax(abi.GC_F64, FAKE, FAKE + (1 << 20), shape(8, 8, 8), float("inf"), -1, s,
                          None),
    lambda s: abi.gc_hmax(abi.GC_U8, FAKE, FAKE + (1 << 20), shape(8, 8, 8), 2.5, -1, s, None),
    # negative erosion size
    lambda s: abi.gc_open_by_reconstruction(abi.GC_U8, FAKE, FAKE + (1 << 20), shape(8, 8, 8), -1,
                                            -1, s, None),
    # null pointers, pitch < width, unknown dtype
    lambda s: abi.gc_hfill(abi.GC_U8, None, FAKE, shape(8, 8, 8), -1, s, None),
    lambda s: abi.gc_raobj(abi.GC_U8, FAKE, None, shape(8, 8, 8), -1, s, None),
    lambda s: abi.gc_raobj(abi.GC_F32, FAKE, FAKE + (1 << 20), shape(8, 8, 7), -1, s, None),
    lambda s: abi.gc_hfill(5, FAKE, FAKE + (1 << 20), shape(8, 8, 8), -1, s, None),
])
def test_operator_invalid_arguments(call):
    s = _steps()
    assert call(ctypes.byref(s)) == abi.GC_ERR_INVALID_ARG
    assert s.value == 0 or s.value == 123
    assert abi.last_error() != ""


def test_operator_aliasing_and_empty():
    s = _steps()
    sh = shape(100, 100, 128)
    # out == f, and out overlapping f's last row: f is the reconstruction's mask
    assert abi.gc_hfill(abi.GC_U8, FAKE, FAKE, sh, -1, ctypes.byref(s), None) == abi.GC_ERR_ALIAS
    assert abi.gc_dome(abi.GC_F32, FAKE, FAKE + 4 * 99 * 128, sh, 1.0, -1, ctypes.byref(s),
                       None) == abi.GC_ERR_ALIAS
    # empty images: nothing to do, no device access
    for fn in ("gc_hfill", "gc_raobj"):
        s = _steps()
        assert getattr(abi, fn)(abi.GC_F64, FAKE, FAKE, shape(0, 5, 1), -1, ctypes.byref(s),
                                None) == abi.GC_OK
        assert s.value == 0
    assert abi.gc_hmax(abi.GC_U8, None, None, shape(7, 0, 7), 3.0, -1, None, None) == abi.GC_OK
    assert abi.gc_open_by_reconstruction(abi.GC_U8, FAKE, FAKE, shape(0, 0, 0), 2, -1, None,
                                         None) == abi.GC_OK


def test_quasi_distance_validation():
    sh = shape(64, 32, 64)
    n1, n2 = ctypes.c_int64(5), ctypes.c_int64(5)
    q = abi.gc_quasi_distance
    assert q(abi.GC_U8, None, FAKE, None, sh, 1, ctypes.byref(n1), ctypes.byref(n2), None) == abi.GC_ERR_INVALID_ARG
    assert n1.value == 0 and n2.value == 0
    assert q(abi.GC_U8, FAKE, None, None, sh, 1, None, None, None) == abi.GC_ERR_INVALID_ARG
    assert q(abi.GC_F32, FAKE, FAKE + (1 << 20) + 2, None, sh, 1, None, None, None) == abi.GC_ERR_INVALID_ARG
    assert q(abi.GC_F32, FAKE, FAKE, None, sh, 1, None, None, None) == abi.GC_ERR_ALIAS
    # dist overlapping the last row of f (f32: 4 bytes per element)
    assert q(abi.GC_F32, FAKE, FAKE + 4 * 31 * 64, None, sh, 0, None, None, None) == abi.GC_ERR_ALIAS
    assert q(abi.GC_U8, FAKE, FAKE + (1 << 20), FAKE + (1 << 20) + 8, sh, 1, None, None,
             None) == abi.GC_ERR_ALIAS
    assert q(9, FAKE, FAKE + (1 << 20), None, sh, 1, None, None, None) == abi.GC_ERR_INVALID_ARG
    assert q(abi.GC_U8, None, None, None, shape(0, 3, 0), 1, ctypes.byref(n1), None, None) == abi.GC_OK


def test_granulometry_and_asf_validation():
    G = (ctypes.c_double * 4)(7, 7, 7, 7)
    sh = shape(16, 16, 16)
    assert abi.gc_granulometry(abi.GC_U8, FAKE, sh, -1, G, None, None) == abi.GC_ERR_INVALID_ARG
    assert abi.gc_granulometry(abi.GC_U8, FAKE, sh, 2, None, None, None) == abi.GC_ERR_INVALID_ARG
    assert abi.gc_granulometry(abi.GC_U8, None, sh, 2, G, None, None) == abi.GC_ERR_INVALID_ARG
    PS = (ctypes.c_double * 3)(7, 7, 7)
    assert abi.gc_granulometry(abi.GC_F32, FAKE, shape(0, 4, 0), 3, G, PS, None) == abi.GC_OK
    assert list(G) == [0, 0, 0, 0] and list(PS) == [0, 0, 0]
    assert abi.gc_asf(abi.GC_U8, FAKE, FAKE + 1, sh, 1, None) == abi.GC_ERR_ALIAS
    assert abi.gc_asf(abi.GC_U8, FAKE, FAKE + (1 << 20), sh, -2, None) == abi.GC_ERR_INVALID_ARG
    assert abi.gc_asf(abi.GC_U8, None, None, shape(0, 0, 0), 2, None) == abi.GC_OK


def test_validate_values_validation():
    v = abi.gc_validate_values
    sh = shape(16, 8, 16)
    assert v(abi.GC_F32, None, sh, 1, None) == abi.GC_ERR_INVALID_ARG
    assert "null" in abi.last_error()
    assert v(9, FAKE, sh, 1, None) == abi.GC_ERR_INVALID_ARG
    assert v(abi.GC_F64, FAKE, shape(16, 8, 15), 0, None) == abi.GC_ERR_INVALID_ARG   # pitch < width
    # nothing to scan: u8 holds no NaN or infinity, empty images hold nothing
    assert v(abi.GC_U8, FAKE, sh, 0, None) == abi.GC_OK
    assert v(abi.GC_F32, None, shape(0, 5, 0), 0, None) == abi.GC_OK


def test_noalloc_chain_refusals():
    """The chain that allocates nothing validates like the geodesic chains
    and refuses images beyond its 16 MiB array before any HIP call."""
    far = 1 << 30
    # an unknown op, negative steps, a null mask
    assert abi.gc_geodesic_chain_noalloc(abi.GC_U8, 5, FAKE, FAKE + far, FAKE + 2 * far,
                                         shape(8, 8, 8), 1, None) == abi.GC_ERR_INVALID_ARG
    assert abi.gc_geodesic_chain_noalloc(abi.GC_U8, abi.GC_DILATE, FAKE, FAKE + far, FAKE + 2 * far,
                                         shape(8, 8, 8), -1, None) == abi.GC_ERR_INVALID_ARG
    assert abi.gc_geodesic_chain_noalloc(abi.GC_U8, abi.GC_ERODE, FAKE, None, FAKE + 2 * far,
                                         shape(8, 8, 8), 1, None) == abi.GC_ERR_INVALID_ARG
    # out on the mask
    assert abi.gc_geodesic_chain_noalloc(abi.GC_F32, abi.GC_DILATE, FAKE, FAKE + far, FAKE + far,
                                         shape(8, 8, 8), 1, None) == abi.GC_ERR_ALIAS
    # extents: 4096 x 4096 u8 is exactly 16 MiB; one more row, or f32 of the same
    # shape, or a pitch that spreads the rows out, is too large
    assert abi.gc_geodesic_chain_noalloc(abi.GC_U8, abi.GC_DILATE, FAKE, FAKE + far, FAKE + 2 * far,
                                         shape(4096, 4097, 4096), 3, None) == abi.GC_ERR_UNSUPPORTED
    assert "16777216" in abi.last_error()
    assert abi.gc_geodesic_chain_noalloc(abi.GC_F32, abi.GC_ERODE, FAKE, FAKE + far, FAKE + 2 * far,
                                         shape(2048, 2049, 2048), 3, None) == abi.GC_ERR_UNSUPPORTED
    assert abi.gc_geodesic_chain_noalloc(abi.GC_F64, abi.GC_DILATE, FAKE, FAKE + far, FAKE + 2 * far,
                                         shape(100, 2049, 1024), 3, None) == abi.GC_ERR_UNSUPPORTED
    # empty images succeed without touching the device
    assert abi.gc_geodesic_chain_noalloc(abi.GC_U8, abi.GC_DILATE, None, None, None,
                                         shape(0, 5, 0), 3, None) == abi.GC_OK


def test_batch_chain_refusals():
    far = 1 << 30
    s = shape(10, 10, 10)
    # stride below the image span, too many images, negative count, null mask
    assert abi.gc_geodesic_chain_batch(abi.GC_U8, abi.GC_DILATE, FAKE, FAKE + far, FAKE + 2 * far, s, 2, 50,
                                       3, None) == abi.GC_ERR_INVALID_ARG
    assert abi.gc_geodesic_chain_batch(abi.GC_U8, abi.GC_DILATE, FAKE, FAKE + far, FAKE + 2 * far, s, 70000,
                                       100, 3, None) == abi.GC_ERR_UNSUPPORTED
    assert abi.gc_geodesic_chain_batch(abi.GC_F32, abi.GC_ERODE, FAKE, FAKE + far, FAKE + 2 * far, s, -1,
                                       100, 3, None) == abi.GC_ERR_INVALID_ARG
    assert abi.gc_geodesic_chain_batch(abi.GC_F64, abi.GC_ERODE, FAKE, None, FAKE + 2 * far, s, 2,
                                       100, 3, None) == abi.GC_ERR_INVALID_ARG
    # out overlapping the second image's mask
    assert abi.gc_geodesic_chain_batch(abi.GC_U8, abi.GC_DILATE, FAKE, FAKE + far, FAKE + far + 150, s, 2,
                                       100, 3, None) == abi.GC_ERR_ALIAS
    # empty batches succeed without touching the device
    assert abi.gc_geodesic_chain_batch(abi.GC_U8, abi.GC_DILATE, None, None, None, s, 0, 0, 3,
                                       None) == abi.GC_OK


def test_struct_layouts_match_the_c_header(tmp_path):
    """The ctypes records have the size and field offsets that a C compiler
    gives the header's structs (compiled with gcc against include/geochain.h,
    which must also be valid C)."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    structs = {"gc_shape": abi.gc_shape, "gc_item": abi.gc_item, "gc_tune_entry": abi.gc_tune_entry}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "geochain.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'    printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'    printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        name, key, value = line.split()
        got[(name, key)] = int(value)
    for name, cls in structs.items():
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert got[(name, field)] == getattr(cls, field).offset, (name, field)
