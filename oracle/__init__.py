"""CPU oracle for chains of elementary 3x3 geodesic dilations / erosions
and the reconstruction-based operators built on them.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg.  The GPU library never imports or calls it.

Thin ctypes front end over ``oracle.c`` (plain C, built by ``oracle/build.py``).
Images are 2-D numpy arrays (rows = y, columns = x) of uint8, float32 or
float64; they are converted exactly to float64 for the C code and the
results are converted back to the input dtype, which is exact because
min/max only select existing values (Section 2, Eq. 1-5).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

DILATE = 0
ERODE = 1
CODE_MASK = 9

_P_D = ctypes.POINTER(ctypes.c_double)
_P_U8 = ctypes.POINTER(ctypes.c_uint8)
_I64 = ctypes.c_int64


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_threads.restype = None
    lib.oracle_max_threads.argtypes = []
    lib.oracle_max_threads.restype = ctypes.c_int
    lib.oracle_step.argtypes = [ctypes.c_int, _P_D, _P_D, _P_D, _I64, _I64]
    lib.oracle_step.restype = _I64
    lib.oracle_chain.argtypes = [ctypes.c_int, _P_D, _P_D, _P_D, _I64, _I64, _I64]
    lib.oracle_chain.restype = ctypes.c_int
    lib.oracle_reconstruct.argtypes = [ctypes.c_int, _P_D, _P_D, _P_D, _I64, _I64, _I64,
                                       ctypes.POINTER(_I64)]
    lib.oracle_reconstruct.restype = ctypes.c_int
    lib.oracle_chain_codes.argtypes = [ctypes.c_int, _P_D, _P_D, _P_D, _P_U8, _I64, _I64, _I64]
    lib.oracle_chain_codes.restype = ctypes.c_int
    lib.oracle_chain_grad.argtypes = [_P_U8, _P_D, _P_D, _P_D, _I64, _I64, _I64]
    lib.oracle_chain_grad.restype = ctypes.c_int
    _lib = lib
    return lib


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def _op(op) -> int:
    if op in (DILATE, "dilate", "dilation"):
        return DILATE
    if op in (ERODE, "erode", "erosion"):
        return ERODE
    raise ValueError(f"unknown op {op!r}")


def _as_f64(a):
    a = np.asarray(a)
    if a.ndim != 2:
        raise ValueError("images are 2-D (rows, columns)")
    if a.dtype not in (np.uint8, np.float32, np.float64):
        raise TypeError(f"unsupported dtype {a.dtype}")
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, t=_P_D):
    return a.ctypes.data_as(t) if a is not None else None


def _back(a64, dtype):
    out = a64.astype(dtype)
    # min/max select existing values, so the round trip must be exact.
    assert np.array_equal(out.astype(np.float64), a64)
    return out


def step(op, f, m=None):
    """One elementary step delta_1^m / eps_1^m (plain delta_1 / eps_1 if m is None)."""
    f64 = _as_f64(f)
    m64 = _as_f64(m) if m is not None else None
    if m64 is not None and m64.shape != f64.shape:
        raise ValueError("marker and mask shapes differ")
    out = np.empty_like(f64)
    Y, X = f64.shape
    _load().oracle_step(_op(op), _ptr(f64), _ptr(m64), _ptr(out), X, Y)
    return _back(out, np.asarray(f).dtype)


def chain(op, f, n, m=None):
    """n-fold composition of the elementary step (Eq. 4); n = 0 is a copy."""
    f64 = _as_f64(f)
    m64 = _as_f64(m) if m is not None else None
    if m64 is not None and m64.shape != f64.shape:
        raise ValueError("marker and mask shapes differ")
    if n < 0:
        raise ValueError("n must be >= 0")
    out = np.empty_like(f64)
    Y, X = f64.shape
    rc = _load().oracle_chain(_op(op), _ptr(f64), _ptr(m64), _ptr(out), X, Y, int(n))
    if rc != 0:
        raise MemoryError("oracle_chain failed")
    return _back(out, np.asarray(f).dtype)


def reconstruct(op, f, m, max_steps=-1):
    """Reconstruction (Eq. 5).  Returns (result, steps_changed, converged)."""
    f64 = _as_f64(f)
    m64 = _as_f64(m)
    if m64.shape != f64.shape:
        raise ValueError("marker and mask shapes differ")
    out = np.empty_like(f64)
    Y, X = f64.shape
    steps = _I64(0)
    rc = _load().oracle_reconstruct(_op(op), _ptr(f64), _ptr(m64), _ptr(out), X, Y,
                                    int(max_steps), ctypes.byref(steps))
    if rc < 0:
        raise MemoryError("oracle_reconstruct failed")
    return _back(out, np.asarray(f).dtype), int(steps.value), rc == 0


def chain_codes(op, f, n, m=None):
    """Forward chain plus the per-step source code of every pixel.

    Returns (result, codes) with codes of shape (n, Y, X), uint8: 0..8 is the
    first extremal neighbour in raster (dy, dx) order, 9 means the mask won.
    """
    f64 = _as_f64(f)
    m64 = _as_f64(m) if m is not None else None
    Y, X = f64.shape
    out = np.empty_like(f64)
    codes = np.empty((int(n), Y, X), dtype=np.uint8)
    rc = _load().oracle_chain_codes(_op(op), _ptr(f64), _ptr(m64), _ptr(out),
                                    _ptr(codes, _P_U8), X, Y, int(n))
    if rc != 0:
        raise MemoryError("oracle_chain_codes failed")
    return _back(out, np.asarray(f).dtype), codes


def chain_grad(codes, g_out):
    """Reverse pass by scattering.  Returns (grad_marker, grad_mask), float64."""
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    g64 = _as_f64(g_out)
    n, Y, X = codes.shape
    if g64.shape != (Y, X):
        raise ValueError("gradient shape differs from the codes")
    gf = np.empty_like(g64)
    gm = np.empty_like(g64)
    rc = _load().oracle_chain_grad(_ptr(codes, _P_U8), _ptr(g64), _ptr(gf), _ptr(gm),
                                   X, Y, n)
    if rc != 0:
        raise MemoryError("oracle_chain_grad failed")
    return gf, gm


def chain_vjp(op, f, m, n, g_out):
    """Gradient of sum(g_out * chain(op, f, n, m)) w.r.t. (f, m), float64."""
    _, codes = chain_codes(op, f, n, m)
    return chain_grad(codes, g_out)


# --------------------------------------------------------------------------
# Reconstruction-based operators (Section 2, Eq. 6-12), composed from the
# reconstruction above and pixelwise arithmetic done in the image's dtype:
#   - uint8 differences saturate at 0 (the paper leaves f - h undefined for
#     8-bit images; the saturating reading keeps markers inside [0, 255]);
#   - float32 / float64 differences are one IEEE subtraction in that dtype,
#     with h first rounded to the dtype;
#   - the border B of an image is its first and last row and column;
#   - every operator returns (image, steps_changed, converged) of its one
#     reconstruction; with a step cap that is reached, the operator is formed
#     from the capped chain.
# --------------------------------------------------------------------------
def _check_image(f):
    f = np.asarray(f)
    _as_f64(f)
    return f


def _h_in_dtype(dtype, h):
    h = float(h)
    if not np.isfinite(h) or h < 0:
        raise ValueError("h must be finite and >= 0")
    if np.dtype(dtype) == np.uint8:
        if h != int(h):
            raise ValueError("h must be an integer for uint8 images")
        return np.uint8(min(int(h), 255))
    return np.dtype(dtype).type(h)


def _sub_in_dtype(a, b):
    """a - b in a's dtype: uint8 saturates at 0, floats round once."""
    if a.dtype == np.uint8:
        d = a.astype(np.int16) - np.asarray(b).astype(np.int16)
        return np.maximum(d, 0).astype(np.uint8)
    return np.subtract(a, b, dtype=a.dtype)


def _border_marker(f, inner):
    """f on the border B, the constant inner everywhere else (Eq. 9, 11)."""
    m = np.full_like(f, inner)
    m[0, :] = f[0, :]
    m[-1, :] = f[-1, :]
    m[:, 0] = f[:, 0]
    m[:, -1] = f[:, -1]
    return m


def hmax(f, h, max_steps=-1):
    """H-maxima (Eq. 6): reconstruction by dilation of f - h under f."""
    f = _check_image(f)
    return reconstruct(DILATE, _sub_in_dtype(f, _h_in_dtype(f.dtype, h)), f, max_steps)


def dome(f, h, max_steps=-1):
    """Dome extraction (Eq. 7): f - HMAX_h(f)."""
    f = _check_image(f)
    r, steps, conv = hmax(f, h, max_steps)
    return _sub_in_dtype(f, r), steps, conv


def hfill(f, max_steps=-1):
    """Hole filling (Eq. 8-9): reconstruction by erosion, above the mask f,
    of the marker that equals f on the border and max f inside."""
    f = _check_image(f)
    if f.size == 0:
        return f.copy(), 0, True
    return reconstruct(ERODE, _border_marker(f, f.max()), f, max_steps)


def raobj(f, max_steps=-1):
    """Removal of border objects (Eq. 10-11): f minus the reconstruction by
    dilation, under f, of the marker that equals f on the border and min f
    inside."""
    f = _check_image(f)
    if f.size == 0:
        return f.copy(), 0, True
    r, steps, conv = reconstruct(DILATE, _border_marker(f, f.min()), f, max_steps)
    return _sub_in_dtype(f, r), steps, conv


def open_by_reconstruction(f, s, max_steps=-1):
    """Opening by reconstruction (Eq. 12): reconstruction by dilation, under
    f, of eps_s(f) = s plain 3x3 erosions of f (Eq. 4 without a mask)."""
    f = _check_image(f)
    if s < 0:
        raise ValueError("s must be >= 0")
    return reconstruct(DILATE, chain(ERODE, f, int(s)), f, max_steps)


def quasi_distance(f):
    """Quasi-distance transform (Eq. 13-15, Algorithm 6).

    Returns (d_l1, d, r, erosion_steps, eta_steps):
      - plain erosions eps_j(f) = eps_1(eps_{j-1}(f)) (Eq. 4 without a mask)
        are applied until one changes nothing, after which every residual is
        0; erosion_steps counts the ones that changed a pixel;
      - r = the largest residual eps_{j-1}(f) - eps_j(f) over j, in f's
        dtype, and d (int32) = the first j that reaches it, 0 where every
        residual is 0 (a later j replaces it only if its residual is
        strictly larger);
      - d_l1 (int32) = eta applied to d until it stops changing, with
        eta(g)(p) = eps_1(g)(p) + 1 where g(p) - eps_1(g)(p) > 1, else g(p)
        (Eq. 14-15); eta_steps counts the applications that changed a pixel.
    """
    f = _check_image(f)
    r = np.zeros_like(f)
    d = np.zeros(f.shape, dtype=np.int32)
    cur = f
    j = 0
    while f.size:
        nxt = step(ERODE, cur)
        if np.array_equal(nxt, cur):
            break
        j += 1
        res = _sub_in_dtype(cur, nxt)   # an erosion never raises a pixel
        upd = res > r
        r[upd] = res[upd]
        d[upd] = j
        cur = nxt
    g = d.astype(np.float64)
    eta = 0
    while f.size:
        e = step(ERODE, g)
        new = np.where(g - e > 1, e + 1, g)
        if np.array_equal(new, g):
            break
        eta += 1
        g = new
    return g.astype(np.int32), d, r, j, eta


def opening(f, s):
    """gamma_s(f) = delta_s(eps_s(f)): s plain erosions, then s plain
    dilations (Eq. 16)."""
    return chain(DILATE, chain(ERODE, f, int(s)), int(s))


def closing(f, s):
    """phi_s(f) = eps_s(delta_s(f)) (Eq. 19)."""
    return chain(ERODE, chain(DILATE, f, int(s)), int(s))


def granulometry(f, s_max):
    """Granulometric function G_s(f) = sum over P of gamma_s(f), s = 0..s_max
    (Eq. 17; gamma_0 = f), each sum exactly rounded to float64 (math.fsum),
    and the pattern spectrum PS_s = G_s - G_{s+1}, s = 0..s_max-1 (Eq. 18)."""
    import math
    f = _check_image(f)
    if s_max < 0:
        raise ValueError("s_max must be >= 0")
    G = np.array([math.fsum(opening(f, s).astype(np.float64).ravel()) for s in range(int(s_max) + 1)])
    return G, G[:-1] - G[1:]


def asf(f, s_max):
    """Alternating sequential filter starting with an opening (Eq. 20):
    phi_s(gamma_s(... phi_1(gamma_1(f)))) up to s = s_max; s_max = 0 is f."""
    f = _check_image(f)
    if s_max < 0:
        raise ValueError("s_max must be >= 0")
    g = f.copy()
    for s in range(1, int(s_max) + 1):
        g = closing(opening(g, s), s)
    return g
