"""MI355X (gfx950) implementation of AIWC's trace-characterization hot path
(Johnston & Milthorpe, arXiv 1805.04207): HIP kernels behind the C ABI of
include/aiwc.h, with a thin ctypes binding (aiwc.py)."""
from .aiwc import (AiwcError, Context, Metrics, Trace, load_library,  # noqa: F401
                   SIZING_BOUND, SIZING_HEURISTIC, SIZING_LEARNED,
                   AUTOTUNE_OFF, AUTOTUNE_CACHED, AUTOTUNE_SEARCH,
                   BRANCH_ZERO_HISTORY, BRANCH_GLOBAL_HISTORY, BRANCH_PATTERN_ENTROPY)
from .host import device_trace, host_to_device  # noqa: F401
