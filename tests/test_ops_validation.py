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
