"""MI355X (gfx950) Convergent-Born-Series operator: HIP kernels behind a C ABI.

The package holds the HIP sources (csrc/), the in-tree built libcbs.so, the
ctypes binding (cbs.py) and its build script (build.py).
"""
from .cbs import (  # noqa: F401
    BornResidualLoss, CbsError, Plan, born_residual_loss, load, pack, unpack, offsets,
    SUPPORTED_SIZES, CBS_C64, CBS_C128,
)
