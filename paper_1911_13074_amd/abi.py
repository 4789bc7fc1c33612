"""ctypes binding of the C ABI in include/geochain.h.

Every function keeps the C name and signature; this module only loads the
library and declares argument types.  It never falls back to anything: if
libgeochain.so is missing, importing the names raises.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# GEOCHAIN_LIB names another build of the same library (the tests load a
# host-sanitizer build through it); by default the in-tree build.
LIB_PATH = os.environ.get("GEOCHAIN_LIB") or os.path.join(_HERE, "libgeochain.so")

GC_U8, GC_F32, GC_F64 = 0, 1, 2
GC_DILATE, GC_ERODE = 0, 1

GC_OK = 0
GC_ERR_INVALID_ARG = -1
GC_ERR_UNSUPPORTED = -2
GC_ERR_ALIAS = -3
GC_ERR_NO_MEMORY = -4
GC_ERR_HIP = -5
GC_ERR_NOT_CONVERGED = -6


class gc_shape(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int64), ("height", ctypes.c_int64), ("pitch", ctypes.c_int64)]


class gc_item(ctypes.Structure):
    _fields_ = [("marker", ctypes.c_void_p), ("mask", ctypes.c_void_p), ("out", ctypes.c_void_p),
                ("shape", gc_shape), ("n_steps", ctypes.c_int64)]


GC_TUNE_FAMILIES = 5


class gc_tune_entry(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("op", ctypes.c_int32), ("geodesic", ctypes.c_int32),
                ("log2_width", ctypes.c_int32), ("log2_height", ctypes.c_int32), ("best_tile", ctypes.c_int32),
                ("k", ctypes.c_int32 * GC_TUNE_FAMILIES), ("rate", ctypes.c_double * GC_TUNE_FAMILIES)]


class GeochainError(RuntimeError):
    def __init__(self, status, func, detail):
        self.status = status
        super().__init__(f"{func}: {status_string(status)} ({detail})")


_VP = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_P_I64 = ctypes.POINTER(ctypes.c_int64)
_DT = ctypes.c_int  # gc_dtype / gc_op are C enums (int)

# name -> (restype, argtypes); mirrors include/geochain.h
SIGNATURES = {
    "gc_version": (ctypes.c_int, []),
    "gc_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "gc_last_error": (ctypes.c_char_p, []),
    "gc_geodesic_dilate_chain": (ctypes.c_int, [_DT, _VP, _VP, _VP, gc_shape, _I64, _VP]),
    "gc_geodesic_erode_chain": (ctypes.c_int, [_DT, _VP, _VP, _VP, gc_shape, _I64, _VP]),
    "gc_geodesic_chain_batch": (ctypes.c_int, [_DT, _DT, _VP, _VP, _VP, gc_shape, _I32, _I64, _I64, _VP]),
    "gc_geodesic_chain_noalloc": (ctypes.c_int, [_DT, _DT, _VP, _VP, _VP, gc_shape, _I64, _VP]),
    "gc_dilate_chain": (ctypes.c_int, [_DT, _VP, _VP, gc_shape, _I64, _VP]),
    "gc_erode_chain": (ctypes.c_int, [_DT, _VP, _VP, gc_shape, _I64, _VP]),
    "gc_reconstruct_by_dilation": (ctypes.c_int, [_DT, _VP, _VP, _VP, gc_shape, _I64, _P_I64, _VP]),
    "gc_reconstruct_by_erosion": (ctypes.c_int, [_DT, _VP, _VP, _VP, gc_shape, _I64, _P_I64, _VP]),
    "gc_hmax": (ctypes.c_int, [_DT, _VP, _VP, gc_shape, ctypes.c_double, _I64, _P_I64, _VP]),
    "gc_dome": (ctypes.c_int, [_DT, _VP, _VP, gc_shape, ctypes.c_double, _I64, _P_I64, _VP]),
    "gc_hfill": (ctypes.c_int, [_DT, _VP, _VP, gc_shape, _I64, _P_I64, _VP]),
    "gc_raobj": (ctypes.c_int, [_DT, _VP, _VP, gc_shape, _I64, _P_I64, _VP]),
    "gc_open_by_reconstruction": (ctypes.c_int, [_DT, _VP, _VP, gc_shape, _I64, _I64, _P_I64, _VP]),
    "gc_quasi_distance": (ctypes.c_int, [_DT, _VP, _VP, _VP, gc_shape, _I32, _P_I64, _P_I64, _VP]),
    "gc_granulometry": (ctypes.c_int, [_DT, _VP, gc_shape, _I32, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double), _VP]),
    "gc_asf": (ctypes.c_int, [_DT, _VP, _VP, gc_shape, _I32, _VP]),
    "gc_set_tuning": (ctypes.c_int, [_I32, _I32]),
    "gc_set_window_path": (ctypes.c_int, [_I32]),
    "gc_validate_values": (ctypes.c_int, [_DT, _VP, gc_shape, _I32, _VP]),
    "gc_plan_create": (ctypes.c_int, [_DT, _DT, ctypes.POINTER(gc_item), _I32,
                                      ctypes.POINTER(ctypes.c_void_p)]),
    "gc_plan_launch": (ctypes.c_int, [_VP, _VP]),
    "gc_plan_status": (ctypes.c_int, [_VP]),
    "gc_plan_steps": (ctypes.c_int, [_VP, _P_I64]),
    "gc_plan_info": (ctypes.c_int, [_VP, _P_I64, _P_I64, ctypes.POINTER(_I32),
                                    ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    "gc_plan_destroy": (ctypes.c_int, [_VP]),
    "gc_plan_tune": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_double)]),
    "gc_autotune": (ctypes.c_int, [_DT, _DT, _I32, _I64, _I64, ctypes.POINTER(_I32),
                                   ctypes.POINTER(_I32)]),
    "gc_autotune_clear": (ctypes.c_int, []),
    "gc_autotune_export": (ctypes.c_int, [ctypes.POINTER(gc_tune_entry), _I32, ctypes.POINTER(_I32)]),
    "gc_autotune_import": (ctypes.c_int, [ctypes.POINTER(gc_tune_entry), _I32]),
    "gc_geodesic_chain_fwd_codes": (ctypes.c_int, [_DT, _DT, _VP, _VP, _VP, _VP, gc_shape, _I32, _I64,
                                                   _I64, _VP]),
    "gc_geodesic_chain_bwd": (ctypes.c_int, [_DT, _DT, _VP, _VP, _VP, _VP, gc_shape, _I32, _I64, _I64, _VP]),
    "gc_geodesic_chain_fwd_sources": (ctypes.c_int, [_DT, _DT, _VP, _VP, _VP, _VP, gc_shape, _I32, _I64, _I64, _VP]),
    "gc_geodesic_chain_bwd_sources": (ctypes.c_int, [_DT, _VP, _VP, _VP, _VP, gc_shape, _I32, _I64, _VP]),
    "gc_profile_enable": (ctypes.c_int, [ctypes.c_int]),
    "gc_profile_read": (ctypes.c_int, [ctypes.POINTER(ctypes.c_double), _P_I64, _P_I64]),
}

_lib = None


def load():
    """Load libgeochain.so (raises OSError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise OSError(f"{LIB_PATH} is missing: build it with paper_1911_13074_amd/build.py "
                      "(or __graft_entry__.build()); there is no fallback path")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def status_string(status: int) -> str:
    return load().gc_status_string(int(status)).decode()


def last_error() -> str:
    return load().gc_last_error().decode()


def check(status: int, func: str) -> int:
    if status != GC_OK:
        raise GeochainError(status, func, last_error())
    return status


def __getattr__(name):
    if name in SIGNATURES:
        return getattr(load(), name)
    raise AttributeError(name)
