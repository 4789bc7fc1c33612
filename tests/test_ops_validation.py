"""Host-side checks of the gradient wrappers: tensors whose layout disagrees
with the one shape, pitch and image stride the C ABI receives are refused
with ValueError/TypeError before any pointer reaches the library (CPU
tensors: the layout checks run before the device check)."""
import ctypes

import pytest
import torch

import paper_1911_13074_amd as gc
from paper_1911_13074_amd import abi


def f32(*shape):
    return torch.zeros(shape, dtype=torch.float32)


@pytest.mark.parametrize("make,msg", [
    (lambda: gc.geodesic_chain_bwd("dilate", torch.zeros((1, 3, 8, 9), dtype=torch.uint8), f32(8, 9),
                                   torch.zeros((8, 9), dtype=torch.float64)), "shape, dtype and device"),
    (lambda: gc.geodesic_chain_bwd("dilate", torch.zeros((1, 3, 8, 9), dtype=torch.uint8), f32(8, 9),
                                   f32(8, 10)), "shape, dtype and device"),
    (lambda: gc.geodesic_chain_bwd("dilate", torch.zeros((1, 3, 8, 9), dtype=torch.uint8), f32(8, 9),
                                   f32(9, 8).t()), "strides differ"),
    (lambda: gc.geodesic_chain_bwd("dilate", torch.zeros((1, 3, 8, 8), dtype=torch.uint8), f32(8, 9),
                                   f32(8, 9)), "codes must be uint8 of shape"),
    (lambda: gc.geodesic_chain_bwd("dilate", torch.zeros((1, 3, 8, 9), dtype=torch.int32), f32(8, 9),
                                   f32(8, 9)), "codes must be uint8"),
    (lambda: gc.geodesic_chain_bwd("dilate", torch.zeros((2, 3, 8, 9), dtype=torch.uint8), f32(8, 9),
                                   f32(8, 9)), "codes must be uint8 of shape"),
    (lambda: gc.geodesic_chain_bwd("dilate", torch.zeros((1, 3, 9, 8), dtype=torch.uint8).transpose(2, 3),
                                   f32(8, 9), f32(8, 9)), "contiguous"),
    (lambda: gc.geodesic_chain_bwd("dilate", torch.zeros((1, 3, 8, 9), dtype=torch.uint8), f32(8, 9),
                                   f32(8, 9), grad_marker=torch.zeros((8, 9))[:, :9].double()),
     "shape, dtype and device"),
    (lambda: gc.geodesic_chain_bwd("open", torch.zeros((1, 3, 8, 9), dtype=torch.uint8), f32(8, 9),
                                   f32(8, 9)), "op is"),
    (lambda: gc.geodesic_chain_fwd_codes("dilate", f32(8, 9), torch.zeros((8, 9), dtype=torch.float64), 3),
     "shape, dtype and device"),
    (lambda: gc.geodesic_chain_fwd_codes("dilate", f32(2, 8, 9), f32(2, 8, 9), 3, out=f32(1, 8, 9)),
     "shape, dtype and device"),
    (lambda: gc.geodesic_chain_fwd_codes("erode", f32(2, 8, 9), f32(2, 8, 9), 3,
                                         codes=torch.zeros((2, 2, 8, 9), dtype=torch.uint8)),
     "codes must be uint8 of shape"),
    (lambda: gc.geodesic_chain_fwd_codes("erode", f32(8, 9), f32(8, 9), 3,
                                         codes=torch.zeros((1, 3, 8, 9), dtype=torch.float32)),
     "codes must be uint8"),
    (lambda: gc.geodesic_chain_fwd_codes("dilate", f32(8, 9), f32(8, 9), 3), "must be a GPU tensor"),
    (lambda: gc.geodesic_chain_bwd("erode", torch.zeros((1, 3, 8, 9), dtype=torch.uint8), f32(8, 9), f32(8, 9)),
     "must be a GPU tensor"),
])
def test_gradient_wrappers_refuse_mismatched_layouts(make, msg):
    with pytest.raises(ValueError, match=msg):
        make()


def test_gradient_wrappers_refuse_integer_images():
    with pytest.raises(TypeError, match="float32 or float64"):
        gc.geodesic_chain_fwd_codes("dilate", torch.zeros((4, 4), dtype=torch.uint8),
                                    torch.zeros((4, 4), dtype=torch.uint8), 2)


def test_backward_entry_point_checks_op():
    """The C entry point validates op like the forward one (GC_DILATE or
    GC_ERODE), before looking at any pointer."""
    fake = 1 << 40
    sh = abi.gc_shape(8, 8, 8)
    st = abi.gc_geodesic_chain_bwd(abi.GC_F32, 7, fake, fake + (1 << 20), fake + (2 << 20), fake + (3 << 20),
                                   sh, 1, 64, 3, None)
    assert st == abi.GC_ERR_INVALID_ARG and "op" in abi.last_error()
    st = abi.gc_geodesic_chain_fwd_codes(abi.GC_F32, 7, fake, fake + (1 << 20), fake + (2 << 20),
                                         ctypes.c_void_p(fake + (3 << 20)), sh, 1, 64, 3, None)
    assert st == abi.GC_ERR_INVALID_ARG
    # empty batch: valid, nothing to do
    assert abi.gc_geodesic_chain_bwd(abi.GC_F64, abi.GC_ERODE, None, None, None, None, sh, 0, 64, 3,
                                     None) == abi.GC_OK


@pytest.mark.parametrize("make,msg", [
    (lambda: gc.geodesic_chain_fwd_sources("dilate", f32(8, 9), f32(8, 9), 3,
                                           sources=torch.zeros((8, 9), dtype=torch.int64)), "sources must be int32"),
    (lambda: gc.geodesic_chain_fwd_sources("dilate", f32(8, 9), f32(8, 9), 3,
                                           sources=torch.zeros((8, 8), dtype=torch.int32)), "sources must be int32"),
    (lambda: gc.geodesic_chain_fwd_sources("dilate", f32(8, 9), f32(8, 9), 3,
                                           sources=torch.zeros((9, 8), dtype=torch.int32).t()), "strides differ"),
    (lambda: gc.geodesic_chain_fwd_sources("dilate", f32(8, 9), f32(8, 10), 3), "shape, dtype and device"),
    (lambda: gc.geodesic_chain_fwd_sources("open", f32(8, 9), f32(8, 9), 3), "op is"),
    (lambda: gc.geodesic_chain_bwd_sources(torch.zeros((8, 9), dtype=torch.int32), f32(8, 9),
                                           torch.zeros((8, 9), dtype=torch.float64)), "shape, dtype and device"),
    (lambda: gc.geodesic_chain_bwd_sources(torch.zeros((2, 8, 9), dtype=torch.int32), f32(8, 9), f32(8, 9)),
     "sources must be int32"),
    (lambda: gc.geodesic_chain_bwd_sources(torch.zeros((8, 9), dtype=torch.int32), f32(8, 9), f32(8, 9),
                                           grad_marker=f32(9, 8).t()), "strides differ"),
])
def test_source_wrappers_refuse_mismatched_layouts(make, msg):
    with pytest.raises((ValueError, TypeError), match=msg):
        make()


def test_source_entry_points_validate_on_the_host():
    """Null pointers, unknown op, integer dtype, images beyond 2^31 - 1
    elements and images taller than the kernels' grid are refused before any
    HIP call."""
    FAKE = 1 << 40
    far = 1 << 44
    s = abi.gc_shape(9, 8, 9)
    assert abi.gc_geodesic_chain_fwd_sources(abi.GC_F32, abi.GC_DILATE, FAKE, FAKE + far, FAKE + 2 * far, None,
                                             s, 1, 0, 3, None) == abi.GC_ERR_INVALID_ARG
    assert abi.gc_geodesic_chain_fwd_sources(abi.GC_F32, 4, FAKE, FAKE + far, FAKE + 2 * far, FAKE + 3 * far,
                                             s, 1, 0, 3, None) == abi.GC_ERR_INVALID_ARG
    assert abi.gc_geodesic_chain_fwd_sources(abi.GC_U8, abi.GC_DILATE, FAKE, FAKE + far, FAKE + 2 * far,
                                             FAKE + 3 * far, s, 1, 0, 3, None) == abi.GC_ERR_UNSUPPORTED
    big = abi.gc_shape(1 << 16, 1 << 15, 1 << 16)   # 2^31 elements
    assert abi.gc_geodesic_chain_fwd_sources(abi.GC_F32, abi.GC_DILATE, FAKE, FAKE + far, FAKE + 2 * far,
                                             FAKE + 3 * far, big, 1, 0, 3, None) == abi.GC_ERR_UNSUPPORTED
    assert "2^31" in abi.last_error()
    # one row of workgroups per core height: 65535 * 112 rows in float32
    tall = abi.gc_shape(16, 65535 * 112 + 1, 16)
    assert abi.gc_geodesic_chain_fwd_sources(abi.GC_F32, abi.GC_DILATE, FAKE, FAKE + far, FAKE + 2 * far,
                                             FAKE + 3 * far, tall, 1, 0, 3, None) == abi.GC_ERR_UNSUPPORTED
    assert "rows" in abi.last_error()
    assert abi.gc_geodesic_chain_bwd_sources(abi.GC_F64, FAKE, FAKE + far, FAKE + far, FAKE + 2 * far,
                                             s, 1, 0, None) == abi.GC_ERR_ALIAS
    assert abi.gc_geodesic_chain_bwd_sources(abi.GC_F64, None, FAKE + far, FAKE + 2 * far, FAKE + 3 * far,
                                             s, 1, 0, None) == abi.GC_ERR_INVALID_ARG
