"""MI355X (gfx950) library for long chains of elementary 3x3 geodesic
dilations and erosions (Zlaus & Mongus, 2019).

The computation lives in hand-written HIP kernels behind the C ABI of
include/geochain.h (libgeochain.so); this package only marshals torch
tensors to it.
"""
from .abi import GeochainError  # noqa: F401
from .autograd import GeodesicChainFunction, geodesic_chain  # noqa: F401
from .ops import (  # noqa: F401
    BatchPlan,
    asf,
    autotune,
    autotune_clear,
    autotune_load,
    autotune_records,
    autotune_save,
    dilate_chain,
    dome,
    erode_chain,
    geodesic_chain_batch,
    geodesic_chain_bwd,
    geodesic_chain_bwd_sources,
    geodesic_chain_fwd_sources,
    geodesic_chain_fwd_codes,
    geodesic_dilate_chain,
    geodesic_erode_chain,
    geodesic_chain_noalloc,
    granulometry,
    hfill,
    hmax,
    open_by_reconstruction,
    quasi_distance,
    raobj,
    reconstruct_by_dilation,
    reconstruct_by_erosion,
    set_tuning,
    set_window_path,
    validate_values,
)
