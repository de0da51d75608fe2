"""Online FISTA for sparse SAR imaging on MI355X (gfx950).

The hot path lives in libofista.so (HIP kernels behind the C ABI of
include/ofista.h); this package holds its sources (csrc/), the build step
(build.py) and a thin ctypes binding (ofista.py).
"""

from .ofista import (  # noqa: F401
    DICT, KERNEL, LIPSCHITZ, MOMENTUM, PRECISION, STORAGE, OfistaConfig, OfistaError,
    OnlineFista, OnlineFistaFn, check_config, coef_count, lib, make_config, workspace_bytes,
)
