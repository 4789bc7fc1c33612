"""GPU value scan (gc_validate_values): a NaN anywhere, and an infinity when
infinities are not allowed, is found; clean images pass.  Positions cover
the first and last pixel, a ragged tail of the 16-byte chunks, padded
pitches (the padding is not scanned) and both scan paths (aligned chunks
and one element per lane)."""
import numpy as np
import pytest
import torch

import paper_1911_13074_amd as gc

pytestmark = pytest.mark.gpu

SHAPES = [(1, 1), (3, 5), (67, 129), (513, 385)]


def positions(h, w):
    return sorted({(0, 0), (h - 1, w - 1), (h // 2, w // 2), (h - 1, 0), (0, w - 1)})


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("shape", SHAPES)
def test_finds_nan_and_infinity(dtype, shape):
    h, w = shape
    base = torch.rand(shape, dtype=dtype, device="cuda") * 10 - 5
    gc.validate_values(base, allow_inf=False)
    for (y, x) in positions(h, w):
        for bad, is_nan in ((float("nan"), True), (float("inf"), False), (float("-inf"), False)):
            t = base.clone()
            t[y, x] = bad
            if is_nan:
                with pytest.raises(ValueError, match="NaN"):
                    gc.validate_values(t)
            else:
                gc.validate_values(t)              # infinities allowed by default
                with pytest.raises(ValueError, match="infinity"):
                    gc.validate_values(t, allow_inf=False)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_padded_pitch_and_unaligned_view(dtype):
    h, w = 70, 203
    big = torch.full((h, 256), float("nan"), dtype=dtype, device="cuda")
    big[:, :w] = 1.5
    view = big[:, :w]                               # NaNs only in the padding
    gc.validate_values(view, allow_inf=False)
    shifted = big[:, 1:w]                           # rows no longer 16-byte aligned
    gc.validate_values(shifted, allow_inf=False)
    big[h - 1, w - 1] = float("-inf")
    with pytest.raises(ValueError, match="infinity"):
        gc.validate_values(big[:, :w], allow_inf=False)
    with pytest.raises(ValueError, match="infinity"):
        gc.validate_values(big[:, 1:w], allow_inf=False)


def test_u8_and_largest_finite_pass():
    gc.validate_values(torch.randint(0, 256, (64, 64), dtype=torch.uint8, device="cuda"), allow_inf=False)
    for dtype in (torch.float32, torch.float64):
        fi = torch.finfo(dtype)
        t = torch.tensor([[fi.max, -fi.max, fi.tiny, -0.0, 0.0]], dtype=dtype, device="cuda")
        gc.validate_values(t, allow_inf=False)
