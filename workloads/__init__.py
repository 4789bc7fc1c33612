"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests and
the benchmark.

This module holds none of the method's arithmetic: it only draws random
images and builds markers from masks by saturating shifts (input
preparation, not a step of the geodesic chain).  The SIPI test images the
paper measures on (Section 4.2) are not available; blurred uniform noise of
the same size and dtype stands in for them.

Recipe of ``blur(h, w, sigma, seed)``:
  1. u = numpy.random.default_rng(seed).random((h, w))   (float64)
  2. separable Gaussian, radius ceil(4 sigma), normalised weights,
     symmetric-reflect padding (scipy.ndimage.gaussian_filter, truncate=4,
     mode="reflect")
  3. min-max rescale to [0, 255], numpy.rint, clip, uint8
"""
from dataclasses import dataclass, field
from typing import List

import numpy as np
from scipy import ndimage


def blur(h: int, w: int, sigma: float, seed: int) -> np.ndarray:
    u = np.random.default_rng(seed).random((h, w))
    b = ndimage.gaussian_filter(u, sigma=sigma, truncate=4.0, mode="reflect")
    lo, hi = float(b.min()), float(b.max())
    if hi > lo:
        b = (b - lo) * (255.0 / (hi - lo))
    else:
        b = np.zeros_like(b)
    return np.clip(np.rint(b), 0, 255).astype(np.uint8)


def sat_sub(a: np.ndarray, h: int) -> np.ndarray:
    """max(a - h, 0) on uint8 without wrap-around."""
    return np.maximum(a.astype(np.int32) - int(h), 0).astype(np.uint8)


def sat_add(a: np.ndarray, h: int) -> np.ndarray:
    """min(a + h, 255) on uint8 without wrap-around."""
    return np.minimum(a.astype(np.int32) + int(h), 255).astype(np.uint8)


# --------------------------------------------------------------------------
# The five workloads.  Shapes are (rows, columns) = (height, width).
# --------------------------------------------------------------------------

def small_u8(size: int = 256, sigma: float = 4.0, seed: int = 1, h: int = 32):
    """256x256 u8: mask = blur(sigma 4), marker = max(mask - 32, 0)."""
    m = blur(size, size, sigma, seed)
    return sat_sub(m, h), m


def headline_u8_dilation(size: int = 1024, seed: int = 2, h: int = 40):
    """1024x1024 u8: mask = blur(sigma 8), marker = max(mask - 40, 0)."""
    m = blur(size, size, 8.0, seed)
    return sat_sub(m, h), m


def headline_u8_erosion(size: int = 1024, seed: int = 2, h: int = 40):
    """1024x1024 u8: mask = blur(sigma 8), marker = min(mask + 40, 255)."""
    m = blur(size, size, 8.0, seed)
    return sat_add(m, h), m


def operator_u8(size: int = 1024, seed: int = 2, sigma: float = 8.0) -> np.ndarray:
    """1024x1024 u8 input of the reconstruction-based operators: the same
    blurred-noise image as the headline mask (the stand-in for the 1024x1024
    8-bit test image of the paper's operator timings)."""
    return blur(size, size, sigma, seed)


def plain_input(dtype, size: int = 1024):
    """1024x1024 plain-chain input: u8 uniform 0..255 (seed 3), f32 / f64
    uniform [0, 1) (seeds 4 / 5)."""
    dtype = np.dtype(dtype)
    if dtype == np.uint8:
        return np.random.default_rng(3).integers(0, 256, size=(size, size)).astype(np.uint8)
    if dtype == np.float32:
        return np.random.default_rng(4).random((size, size), dtype=np.float32)
    if dtype == np.float64:
        return np.random.default_rng(5).random((size, size))
    raise TypeError(dtype)


@dataclass
class BatchItem:
    marker: np.ndarray
    mask: np.ndarray
    n_steps: int


@dataclass
class Batch:
    items: List[BatchItem] = field(default_factory=list)

    @property
    def px_steps(self) -> int:
        return sum(int(it.mask.size) * int(it.n_steps) for it in self.items)


def batch_u8(count: int = 64, lo: int = 128, hi: int = 2048, n_lo: int = 10,
             n_hi: int = 1500, seed: int = 6, sigma: float = 8.0) -> Batch:
    """Uneven batch: sides U{lo..hi} drawn independently, mask = blur(sigma 8,
    seed 1000 + i), h ~ U{8..64}, marker = max(mask - h, 0), chain length
    U{n_lo..n_hi}."""
    rng = np.random.default_rng(seed)
    out = Batch()
    for i in range(count):
        w = int(rng.integers(lo, hi + 1))
        h_img = int(rng.integers(lo, hi + 1))
        hshift = int(rng.integers(8, 65))
        n = int(rng.integers(n_lo, n_hi + 1))
        m = blur(h_img, w, sigma, 1000 + i)
        out.items.append(BatchItem(sat_sub(m, hshift), m, n))
    return out


def differentiable_f32(batch: int = 16, size: int = 1024, seed: int = 7,
                       grad_seed: int = 8, shift: float = 0.1):
    """B x size x size float32: mask = U[0,1) + 1e-4 N(0,1) jitter, marker =
    mask - 0.1, upstream gradient N(0,1).  Returns (marker, mask, grad)."""
    rng = np.random.default_rng(seed)
    m = rng.random((batch, size, size), dtype=np.float32)
    m = m + (1e-4 * rng.standard_normal((batch, size, size))).astype(np.float32)
    f = m - np.float32(shift)
    g = np.random.default_rng(grad_seed).standard_normal((batch, size, size)).astype(np.float32)
    return f.astype(np.float32), m.astype(np.float32), g


def tie_free(h: int, w: int, seed: int, dtype=np.float64, lo_gap: float = 1.0):
    """Marker / mask pair whose 2*h*w values are all distinct (a shuffled
    arithmetic progression), with marker < mask pixelwise."""
    rng = np.random.default_rng(seed)
    vals = rng.permutation(2 * h * w).astype(np.float64) * lo_gap
    a = vals[: h * w].reshape(h, w)
    b = vals[h * w:].reshape(h, w)
    f = np.minimum(a, b)
    m = np.maximum(a, b)
    return f.astype(dtype), m.astype(dtype)
