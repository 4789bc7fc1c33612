"""Torch-facing calls of the geodesic chain library.

Argument marshalling only: every function checks the tensors, passes their
device pointers, shape, pitch and torch's current HIP stream to the C ABI
(abi.py) and returns.  No step of the method runs here.

Images are 2-D device tensors of dtype uint8, float32 or float64 whose rows
are contiguous (stride(1) == 1); stride(0) is the row pitch.
"""
import ctypes
import json

import torch

from . import abi

_DTYPES = {torch.uint8: abi.GC_U8, torch.float32: abi.GC_F32, torch.float64: abi.GC_F64}


def _dtype_code(t: torch.Tensor) -> int:
    try:
        return _DTYPES[t.dtype]
    except KeyError:
        raise TypeError(f"unsupported dtype {t.dtype}; use uint8, float32 or float64") from None


def _check_image(t: torch.Tensor, name: str) -> None:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must live on a GPU device (got {t.device})")
    if t.dim() != 2:
        raise ValueError(f"{name} must be 2-D (rows, columns), got shape {tuple(t.shape)}")
    if t.size(1) > 1 and t.stride(1) != 1:
        raise ValueError(f"{name} rows must be contiguous (stride(1) == 1)")


def _shape(t: torch.Tensor) -> abi.gc_shape:
    h, w = t.shape
    pitch = t.stride(0) if h > 1 else max(w, 1)
    return abi.gc_shape(w, h, max(pitch, w))


def _same_layout(a: torch.Tensor, b: torch.Tensor, names: str) -> None:
    if a.shape != b.shape or a.dtype != b.dtype or a.device != b.device:
        raise ValueError(f"{names}: shape, dtype and device must match")
    if a.size(0) > 1 and a.stride(0) != b.stride(0):
        raise ValueError(f"{names}: row pitches differ")


def _stream(t: torch.Tensor):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


def _out_like(t: torch.Tensor, out):
    if out is None:
        return torch.empty_like(t, memory_format=torch.contiguous_format) if t.is_contiguous() \
            else torch.empty_strided(t.shape, t.stride(), dtype=t.dtype, device=t.device)
    _check_image(out, "out")
    _same_layout(t, out, "marker/out")
    return out


def _geodesic(fn_name, marker, mask, n_steps, out):
    _check_image(marker, "marker")
    _check_image(mask, "mask")
    _same_layout(marker, mask, "marker/mask")
    out = _out_like(marker, out)
    with torch.cuda.device(marker.device):
        st = getattr(abi, fn_name)(_dtype_code(marker), _ptr(marker), _ptr(mask), _ptr(out),
                                   _shape(marker), int(n_steps), _stream(marker))
    abi.check(st, fn_name)
    return out


def geodesic_dilate_chain(marker, mask, n_steps, out=None):
    """n_steps elementary geodesic dilations min(delta_1(f), mask) (Eq. 3-4)."""
    return _geodesic("gc_geodesic_dilate_chain", marker, mask, n_steps, out)


def geodesic_erode_chain(marker, mask, n_steps, out=None):
    """n_steps elementary geodesic erosions max(eps_1(f), mask) (Eq. 3-4)."""
    return _geodesic("gc_geodesic_erode_chain", marker, mask, n_steps, out)


def geodesic_chain_noalloc(op, marker, mask, n_steps, out):
    """The geodesic chain (Eq. 3-4) through the entry point that allocates
    no device memory: its ping-pong image is the library's fixed per-device
    array (images up to 16 MiB), shared by every such call on the device.
    op is "dilate" or "erode"; out must be given (it may be marker)."""
    _check_image(marker, "marker")
    _check_image(mask, "mask")
    _same_layout(marker, mask, "marker/mask")
    if out is None:
        raise ValueError("out must be given: this entry point is for callers that do not allocate")
    _check_image(out, "out")
    _same_layout(marker, out, "marker/out")
    with torch.cuda.device(marker.device):
        st = abi.gc_geodesic_chain_noalloc(_dtype_code(marker), _op_code(op), _ptr(marker), _ptr(mask),
                                           _ptr(out), _shape(marker), int(n_steps), _stream(marker))
    abi.check(st, "gc_geodesic_chain_noalloc")
    return out


def _plain(fn_name, x, n_steps, out):
    _check_image(x, "input")
    out = _out_like(x, out)
    with torch.cuda.device(x.device):
        st = getattr(abi, fn_name)(_dtype_code(x), _ptr(x), _ptr(out), _shape(x), int(n_steps),
                                   _stream(x))
    abi.check(st, fn_name)
    return out


def dilate_chain(x, n_steps, out=None):
    """n_steps plain 3x3 dilations = one (2n+1)^2 clipped window max (Eq. 2)."""
    return _plain("gc_dilate_chain", x, n_steps, out)


def erode_chain(x, n_steps, out=None):
    """n_steps plain 3x3 erosions = one (2n+1)^2 clipped window min (Eq. 1)."""
    return _plain("gc_erode_chain", x, n_steps, out)


def _reconstruct(fn_name, marker, mask, max_steps, out, allow_not_converged):
    _check_image(marker, "marker")
    _check_image(mask, "mask")
    _same_layout(marker, mask, "marker/mask")
    out = _out_like(marker, out)
    steps = ctypes.c_int64(0)
    with torch.cuda.device(marker.device):
        st = getattr(abi, fn_name)(_dtype_code(marker), _ptr(marker), _ptr(mask), _ptr(out),
                                   _shape(marker), int(max_steps), ctypes.byref(steps),
                                   _stream(marker))
    if st == abi.GC_ERR_NOT_CONVERGED and allow_not_converged:
        return out, int(steps.value), False
    abi.check(st, fn_name)
    return out, int(steps.value), True


def reconstruct_by_dilation(marker, mask, max_steps=-1, out=None, allow_not_converged=False):
    """Reconstruction by dilation (Eq. 5).  Returns (image, steps_changed,
    converged); synchronises the current stream."""
    return _reconstruct("gc_reconstruct_by_dilation", marker, mask, max_steps, out,
                        allow_not_converged)


def reconstruct_by_erosion(marker, mask, max_steps=-1, out=None, allow_not_converged=False):
    """Reconstruction by erosion (Eq. 5).  Returns (image, steps_changed,
    converged); synchronises the current stream."""
    return _reconstruct("gc_reconstruct_by_erosion", marker, mask, max_steps, out,
                        allow_not_converged)


def _operator(fn_name, f, extra, max_steps, out, allow_not_converged):
    _check_image(f, "f")
    out = _out_like(f, out)
    steps = ctypes.c_int64(0)
    with torch.cuda.device(f.device):
        st = getattr(abi, fn_name)(_dtype_code(f), _ptr(f), _ptr(out), _shape(f), *extra,
                                   int(max_steps), ctypes.byref(steps), _stream(f))
    if st == abi.GC_ERR_NOT_CONVERGED and allow_not_converged:
        return out, int(steps.value), False
    abi.check(st, fn_name)
    return out, int(steps.value), True


def hmax(f, h, max_steps=-1, out=None, allow_not_converged=False):
    """H-maxima (Eq. 6): reconstruction by dilation of f - h under f.
    Returns (image, steps_changed, converged); synchronises the stream."""
    return _operator("gc_hmax", f, (float(h),), max_steps, out, allow_not_converged)


def dome(f, h, max_steps=-1, out=None, allow_not_converged=False):
    """Dome extraction (Eq. 7): f - HMAX_h(f)."""
    return _operator("gc_dome", f, (float(h),), max_steps, out, allow_not_converged)


def hfill(f, max_steps=-1, out=None, allow_not_converged=False):
    """Hole filling (Eq. 8-9): reconstruction by erosion of the border
    marker (f on the border, max f inside) above f."""
    return _operator("gc_hfill", f, (), max_steps, out, allow_not_converged)


def raobj(f, max_steps=-1, out=None, allow_not_converged=False):
    """Removal of objects touching the border (Eq. 10-11)."""
    return _operator("gc_raobj", f, (), max_steps, out, allow_not_converged)


def open_by_reconstruction(f, size, max_steps=-1, out=None, allow_not_converged=False):
    """Opening by reconstruction (Eq. 12): reconstruction by dilation of
    size plain erosions of f, under f."""
    return _operator("gc_open_by_reconstruction", f, (int(size),), max_steps, out,
                     allow_not_converged)


def quasi_distance(f, lipschitz=True, with_residual=False):
    """Quasi-distance transform (Eq. 13-15).  Returns (dist, residual,
    erosion_steps, eta_steps): dist is int32 (d_L1 if lipschitz, else the
    discontinuous d of Eq. 13), residual is None unless requested.
    Synchronises the current stream."""
    _check_image(f, "f")
    dist = torch.empty_strided(f.shape, f.stride(), dtype=torch.int32, device=f.device)
    res = torch.empty_strided(f.shape, f.stride(), dtype=f.dtype, device=f.device) if with_residual else None
    n_erode = ctypes.c_int64(0)
    n_eta = ctypes.c_int64(0)
    with torch.cuda.device(f.device):
        st = abi.gc_quasi_distance(_dtype_code(f), _ptr(f), _ptr(dist), _ptr(res) if res is not None else None,
                                   _shape(f), 1 if lipschitz else 0, ctypes.byref(n_erode),
                                   ctypes.byref(n_eta), _stream(f))
    abi.check(st, "gc_quasi_distance")
    return dist, res, int(n_erode.value), int(n_eta.value)


def granulometry(f, s_max):
    """Granulometric function G_s (s = 0..s_max) and pattern spectrum PS_s
    (s = 0..s_max-1) of f (Eq. 16-18), as lists of floats.  Synchronises
    the current stream."""
    _check_image(f, "f")
    s_max = int(s_max)
    G = (ctypes.c_double * (s_max + 1))()
    PS = (ctypes.c_double * max(s_max, 1))()
    with torch.cuda.device(f.device):
        st = abi.gc_granulometry(_dtype_code(f), _ptr(f), _shape(f), s_max, G, PS, _stream(f))
    abi.check(st, "gc_granulometry")
    return list(G), list(PS)[:s_max]


def asf(f, s_max, out=None):
    """Alternating sequential filter phi_s(gamma_s(... phi_1(gamma_1(f))))
    up to s = s_max (Eq. 19-20)."""
    _check_image(f, "f")
    out = _out_like(f, out)
    with torch.cuda.device(f.device):
        st = abi.gc_asf(_dtype_code(f), _ptr(f), _ptr(out), _shape(f), int(s_max), _stream(f))
    abi.check(st, "gc_asf")
    return out


def validate_values(x, allow_inf=True):
    """Raise ValueError if the device image holds a NaN (or, with
    allow_inf=False, an infinity); u8 images always pass.  Synchronises
    the current stream."""
    _check_image(x, "image")
    with torch.cuda.device(x.device):
        st = abi.gc_validate_values(_dtype_code(x), _ptr(x), _shape(x), int(bool(allow_inf)), _stream(x))
    if st == abi.GC_ERR_INVALID_ARG:
        raise ValueError(abi.last_error())
    abi.check(st, "gc_validate_values")


def set_window_path(min_steps: int = 0) -> None:
    """Plain chains of at least min_steps steps run as one separable
    (2n+1)^2 window (0: built-in threshold, -1: never)."""
    abi.check(abi.gc_set_window_path(int(min_steps)), "gc_set_window_path")


def set_tuning(block_steps: int = 0, tile: int = -1) -> None:
    """Override steps per launch and tile family (0 / -1: built-in choice)."""
    abi.check(abi.gc_set_tuning(int(block_steps), int(tile)), "gc_set_tuning")


class BatchPlan:
    """Many independent chains in one persistent, graph-recorded launch.

    items: sequence of (marker, mask_or_None, n_steps) or (marker, mask,
    n_steps, out).  All images share one dtype and device; all items are
    geodesic (mask given) or all plain.  n_steps < 0 (geodesic items) runs
    to stability; steps() then gives each item's step count, and launch()
    waits for the result.  The outputs are allocated here when not given.
    launch() replays the recorded graph on the current stream.
    """

    def __init__(self, op, items):
        if op not in ("dilate", "erode"):
            raise ValueError("op is 'dilate' or 'erode'")
        self._plan = None
        self.outs = []
        self._keep = []
        arr = (abi.gc_item * max(len(items), 1))()
        dtype = None
        self.device = None
        for i, it in enumerate(items):
            marker, mask, n = it[0], it[1], int(it[2])
            out = it[3] if len(it) > 3 else None
            _check_image(marker, "marker")
            if mask is not None:
                _check_image(mask, "mask")
                _same_layout(marker, mask, "marker/mask")
            out = _out_like(marker, out)
            if dtype is None:
                dtype, self.device = marker.dtype, marker.device
            elif marker.dtype != dtype or marker.device != self.device:
                raise ValueError("all items share one dtype and device")
            self.outs.append(out)
            self._keep += [marker, mask]
            arr[i].marker = marker.data_ptr()
            arr[i].mask = mask.data_ptr() if mask is not None else None
            arr[i].out = out.data_ptr()
            arr[i].shape = _shape(marker)
            arr[i].n_steps = n
        self.dtype = dtype if dtype is not None else torch.uint8
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device if self.device is not None else torch.cuda.current_device()):
            st = abi.gc_plan_create(_DTYPES[self.dtype], abi.GC_DILATE if op == "dilate" else abi.GC_ERODE,
                                    arr, len(items), ctypes.byref(handle))
        abi.check(st, "gc_plan_create")
        self._plan = handle

    def launch(self):
        dev = self.device if self.device is not None else torch.device("cuda", torch.cuda.current_device())
        with torch.cuda.device(dev):
            stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
            abi.check(abi.gc_plan_launch(self._plan, stream), "gc_plan_launch")
        return self.outs

    def status(self):
        abi.check(abi.gc_plan_status(self._plan), "gc_plan_status")

    def steps(self):
        """Steps of the last launch per item: n_steps for fixed-length items,
        the steps that changed a pixel for run-to-stability items (n < 0)."""
        arr = (ctypes.c_int64 * max(len(self.outs), 1))()
        abi.check(abi.gc_plan_steps(self._plan, arr), "gc_plan_steps")
        return [int(arr[i]) for i in range(len(self.outs))]

    def info(self):
        px, items = ctypes.c_int64(), ctypes.c_int64()
        wgs, tile, k = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        abi.check(abi.gc_plan_info(self._plan, ctypes.byref(px), ctypes.byref(items), ctypes.byref(wgs),
                                   ctypes.byref(tile), ctypes.byref(k)), "gc_plan_info")
        return {"px_steps": px.value, "work_items": items.value, "workgroups": wgs.value,
                "tile": tile.value, "block_steps": k.value}

    def tune(self):
        """Time the launch shapes on scratch images of this batch's shapes
        and rebuild the plan with the fastest; returns its ms per launch."""
        ms = ctypes.c_double()
        dev = self.device if self.device is not None else torch.device("cuda", torch.cuda.current_device())
        with torch.cuda.device(dev):
            torch.cuda.current_stream(dev).synchronize()
            abi.check(abi.gc_plan_tune(self._plan, ctypes.byref(ms)), "gc_plan_tune")
        return ms.value

    def close(self):
        if self._plan is not None:
            abi.gc_plan_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(dtype, op, geodesic, width, height):
    """Time the batch kernel's launch shapes for a size class; the choice
    is used by later plans.  Returns (tile_family, steps_per_block)."""
    code = _DTYPES[dtype] if isinstance(dtype, torch.dtype) else int(dtype)
    tile, k = ctypes.c_int32(), ctypes.c_int32()
    abi.check(abi.gc_autotune(code, abi.GC_DILATE if op == "dilate" else abi.GC_ERODE, int(bool(geodesic)),
                              int(width), int(height), ctypes.byref(tile), ctypes.byref(k)), "gc_autotune")
    return tile.value, k.value


def autotune_clear():
    abi.check(abi.gc_autotune_clear(), "gc_autotune_clear")


_TUNE_FORMAT = "geochain-autotune"
_TUNE_FIELDS = ("dtype", "op", "geodesic", "log2_width", "log2_height", "best_tile")


def autotune_records():
    """The autotuner's table as a list of dicts (one per size class)."""
    count = ctypes.c_int32()
    abi.check(abi.gc_autotune_export(None, 0, ctypes.byref(count)), "gc_autotune_export")
    n = count.value
    arr = (abi.gc_tune_entry * max(n, 1))()
    abi.check(abi.gc_autotune_export(arr, n, ctypes.byref(count)), "gc_autotune_export")
    return [dict({f: getattr(e, f) for f in _TUNE_FIELDS}, k=list(e.k), rate=list(e.rate))
            for e in arr[:min(n, count.value)]]


def autotune_save(path):
    """Write the autotuner's table to a JSON file, for autotune_load in a
    later process."""
    doc = {"format": _TUNE_FORMAT, "version": 1, "families": abi.GC_TUNE_FAMILIES,
           "records": autotune_records()}
    with open(path, "w") as fh:
        json.dump(doc, fh, indent=1)


def autotune_load(path):
    """Add the records of a file that autotune_save wrote to the table
    (replacing those of the same size class).  Raises ValueError for a file
    of another shape; the library checks every value and, on a bad one,
    leaves the table unchanged."""
    with open(path) as fh:
        doc = json.load(fh)
    if not isinstance(doc, dict) or doc.get("format") != _TUNE_FORMAT or doc.get("version") != 1:
        raise ValueError(f"{path}: not an autotune file of this library")
    if doc.get("families") != abi.GC_TUNE_FAMILIES or not isinstance(doc.get("records"), list):
        raise ValueError(f"{path}: records for {doc.get('families')} tile families, this build has "
                         f"{abi.GC_TUNE_FAMILIES}")
    recs = doc["records"]
    arr = (abi.gc_tune_entry * max(len(recs), 1))()
    for i, r in enumerate(recs):
        try:
            for f in _TUNE_FIELDS:
                setattr(arr[i], f, int(r[f]))
            if len(r["k"]) != abi.GC_TUNE_FAMILIES or len(r["rate"]) != abi.GC_TUNE_FAMILIES:
                raise ValueError("one value per tile family")
            for j in range(abi.GC_TUNE_FAMILIES):
                arr[i].k[j] = int(r["k"][j])
                arr[i].rate[j] = float(r["rate"][j])
        except (KeyError, TypeError, ValueError) as exc:
            raise ValueError(f"{path}: record {i}: {exc}") from None
    abi.check(abi.gc_autotune_import(arr, len(recs)), "gc_autotune_import")


def _batch_view(t: torch.Tensor, name: str):
    """(B, H, W) or (H, W) tensor -> (tensor, n_images, image_stride, shape).
    The device is checked separately (_on_gpu), after the layout checks."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dim() == 2:
        t3 = t.unsqueeze(0)
    elif t.dim() == 3:
        t3 = t
    else:
        raise ValueError(f"{name} must be (H, W) or (B, H, W)")
    b, h, w = t3.shape
    if w > 1 and t3.stride(2) != 1:
        raise ValueError(f"{name} rows must be contiguous")
    pitch = t3.stride(1) if h > 1 else max(w, 1)
    stride = t3.stride(0) if b > 1 else (h - 1) * pitch + w if h > 0 else 0
    return t3, b, stride, abi.gc_shape(w, h, max(pitch, w))


_OPS = {"dilate": abi.GC_DILATE, "erode": abi.GC_ERODE}


def _op_code(op) -> int:
    try:
        return _OPS[op]
    except (KeyError, TypeError):
        raise ValueError(f"op is 'dilate' or 'erode', got {op!r}") from None


def _check_batch_like(ref: torch.Tensor, t: torch.Tensor, names: str) -> None:
    """t must have ref's shape, dtype, device and strides (the C ABI takes
    one shape, pitch and image stride for both)."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{names}: expected a torch.Tensor")
    if t.shape != ref.shape or t.dtype != ref.dtype or t.device != ref.device:
        raise ValueError(f"{names}: shape, dtype and device must match "
                         f"({tuple(t.shape)} {t.dtype} {t.device} vs {tuple(ref.shape)} {ref.dtype} {ref.device})")
    # strides of dimensions of size 1 are never used to address memory
    if t.numel() > 0 and any(n > 1 and a != b for n, a, b in zip(t.shape, t.stride(), ref.stride())):
        raise ValueError(f"{names}: strides differ ({t.stride()} vs {ref.stride()})")


def _check_codes(codes, n_images: int, n_steps: int, shape, device) -> None:
    """codes: dense uint8 (n_images, n_steps, height, width) on device."""
    if not isinstance(codes, torch.Tensor):
        raise TypeError("codes must be a torch.Tensor")
    want = (n_images, n_steps, shape.height, shape.width)
    if codes.dtype != torch.uint8 or tuple(codes.shape) != want or codes.device != device:
        raise ValueError(f"codes must be uint8 of shape {want} on {device} "
                         f"(got {codes.dtype} {tuple(codes.shape)} on {codes.device})")
    if not codes.is_contiguous():
        raise ValueError("codes must be contiguous")


def _on_gpu(t: torch.Tensor, name: str) -> None:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor (got {t.device})")


def _check_float_images(*ts):
    for name, t in ts:
        if t.dtype not in (torch.float32, torch.float64):
            raise TypeError(f"{name}: gradients need float32 or float64 images, got {t.dtype}")


def geodesic_chain_fwd_codes(op, marker, mask, n_steps, out=None, codes=None):
    """n_steps geodesic steps that also record each pixel's source per step.

    marker, mask: (H, W) or (B, H, W) float32/float64 with the same layout.
    Returns (out, codes) with codes of shape (B, n_steps, H, W) uint8 (B = 1
    for 2-D inputs).  A given out must have marker's layout; given codes
    must be dense uint8 of that shape on the same device.
    """
    opc = _op_code(op)
    n_steps = int(n_steps)
    _, b, stride, shape = _batch_view(marker, "marker")
    _batch_view(mask, "mask")
    _check_float_images(("marker", marker), ("mask", mask))
    _check_batch_like(marker, mask, "marker/mask")
    if out is not None:
        _check_batch_like(marker, out, "marker/out")
    if codes is not None:
        _check_codes(codes, b, n_steps, shape, marker.device)
    _on_gpu(marker, "marker")
    if out is None:
        out = torch.empty_strided(marker.shape, marker.stride(), dtype=marker.dtype, device=marker.device)
    if codes is None:
        codes = torch.empty((b, n_steps, shape.height, shape.width), dtype=torch.uint8, device=marker.device)
    with torch.cuda.device(marker.device):
        st = abi.gc_geodesic_chain_fwd_codes(_dtype_code(marker), opc, _ptr(marker), _ptr(mask), _ptr(out),
                                             _ptr(codes), shape, b, stride, n_steps, _stream(marker))
    abi.check(st, "gc_geodesic_chain_fwd_codes")
    return out, codes


def geodesic_chain_bwd(op, codes, grad_out, grad_mask, grad_marker=None):
    """Reverse pass over codes (B, n, H, W) recorded by
    geodesic_chain_fwd_codes(op, ...): returns the gradient w.r.t. the state
    before the first step and adds the mask's gradient into grad_mask.
    grad_mask (and a given grad_marker) must have grad_out's layout."""
    opc = _op_code(op)
    _, b, stride, shape = _batch_view(grad_out, "grad_out")
    _check_float_images(("grad_out", grad_out))
    _check_batch_like(grad_out, grad_mask, "grad_out/grad_mask")
    if not isinstance(codes, torch.Tensor) or codes.dim() != 4:
        raise ValueError("codes must be a (B, n_steps, H, W) uint8 tensor")
    n_steps = int(codes.shape[1])
    _check_codes(codes, b, n_steps, shape, grad_out.device)
    if grad_marker is not None:
        _check_batch_like(grad_out, grad_marker, "grad_out/grad_marker")
    _on_gpu(grad_out, "grad_out")
    if grad_marker is None:
        grad_marker = torch.empty_strided(grad_out.shape, grad_out.stride(), dtype=grad_out.dtype,
                                          device=grad_out.device)
    with torch.cuda.device(grad_out.device):
        st = abi.gc_geodesic_chain_bwd(_dtype_code(grad_out), opc, _ptr(codes), _ptr(grad_out),
                                       _ptr(grad_marker), _ptr(grad_mask), shape, b, stride, n_steps,
                                       _stream(grad_out))
    abi.check(st, "gc_geodesic_chain_bwd")
    return grad_marker


def geodesic_chain_batch(op, marker, mask, n_steps, out=None):
    """n_steps geodesic dilations ('dilate') or erosions ('erode') of every
    image of a (B, H, W) batch (or one (H, W) image) under its mask, in one
    launch per block of steps.  mask (and a given out) must have marker's
    layout; out may be marker."""
    opc = _op_code(op)
    _, b, stride, shape = _batch_view(marker, "marker")
    _batch_view(mask, "mask")
    _dtype_code(marker)
    _check_batch_like(marker, mask, "marker/mask")
    if out is not None:
        _check_batch_like(marker, out, "marker/out")
    _on_gpu(marker, "marker")
    if out is None:
        out = torch.empty_strided(marker.shape, marker.stride(), dtype=marker.dtype, device=marker.device)
    with torch.cuda.device(marker.device):
        st = abi.gc_geodesic_chain_batch(_dtype_code(marker), opc, _ptr(marker), _ptr(mask), _ptr(out), shape, b,
                                         stride, int(n_steps), _stream(marker))
    abi.check(st, "gc_geodesic_chain_batch")
    return out


def _check_sources(ref: torch.Tensor, sources, names: str) -> None:
    """sources: int32 with ref's shape, strides and device (the C ABI reads
    them as uint32 with the images' layout)."""
    if not isinstance(sources, torch.Tensor):
        raise TypeError(f"{names}: sources must be a torch.Tensor")
    if sources.dtype != torch.int32 or sources.shape != ref.shape or sources.device != ref.device:
        raise ValueError(f"{names}: sources must be int32 of shape {tuple(ref.shape)} on {ref.device} "
                         f"(got {sources.dtype} {tuple(sources.shape)} on {sources.device})")
    if sources.numel() > 0 and any(n > 1 and a != b for n, a, b in zip(ref.shape, sources.stride(), ref.stride())):
        raise ValueError(f"{names}: sources strides differ ({sources.stride()} vs {ref.stride()})")


def geodesic_chain_fwd_sources(op, marker, mask, n_steps, out=None, sources=None):
    """n_steps geodesic steps that also give each output pixel its source:
    the element offset (y * pitch + x) of the marker pixel, or with the top
    bit set of the mask pixel, whose value it carries.

    marker, mask: (H, W) or (B, H, W) float32/float64 with the same layout.
    Returns (out, sources), sources int32 with marker's layout (the top bit
    makes mask sources negative).
    """
    opc = _op_code(op)
    n_steps = int(n_steps)
    _, b, stride, shape = _batch_view(marker, "marker")
    _batch_view(mask, "mask")
    _check_float_images(("marker", marker), ("mask", mask))
    _check_batch_like(marker, mask, "marker/mask")
    if out is not None:
        _check_batch_like(marker, out, "marker/out")
    if sources is not None:
        _check_sources(marker, sources, "marker/sources")
    _on_gpu(marker, "marker")
    if out is None:
        out = torch.empty_strided(marker.shape, marker.stride(), dtype=marker.dtype, device=marker.device)
    if sources is None:
        sources = torch.empty_strided(marker.shape, marker.stride(), dtype=torch.int32, device=marker.device)
    with torch.cuda.device(marker.device):
        st = abi.gc_geodesic_chain_fwd_sources(_dtype_code(marker), opc, _ptr(marker), _ptr(mask), _ptr(out),
                                               _ptr(sources), shape, b, stride, n_steps, _stream(marker))
    abi.check(st, "gc_geodesic_chain_fwd_sources")
    return out, sources


def geodesic_chain_bwd_sources(sources, grad_out, grad_mask, grad_marker=None):
    """Reverse pass through source ids from geodesic_chain_fwd_sources:
    returns the gradient w.r.t. the state before the first step and adds
    the mask's gradient into grad_mask.  grad_mask, sources (and a given
    grad_marker) must have grad_out's layout."""
    _, b, stride, shape = _batch_view(grad_out, "grad_out")
    _check_float_images(("grad_out", grad_out))
    _check_batch_like(grad_out, grad_mask, "grad_out/grad_mask")
    _check_sources(grad_out, sources, "grad_out/sources")
    if grad_marker is not None:
        _check_batch_like(grad_out, grad_marker, "grad_out/grad_marker")
    _on_gpu(grad_out, "grad_out")
    if grad_marker is None:
        grad_marker = torch.empty_strided(grad_out.shape, grad_out.stride(), dtype=grad_out.dtype,
                                          device=grad_out.device)
    with torch.cuda.device(grad_out.device):
        st = abi.gc_geodesic_chain_bwd_sources(_dtype_code(grad_out), _ptr(sources), _ptr(grad_out),
                                               _ptr(grad_marker), _ptr(grad_mask), shape, b, stride,
                                               _stream(grad_out))
    abi.check(st, "gc_geodesic_chain_bwd_sources")
    return grad_marker
