"""Kinetic maximum-principle bounds and squeeze limiting on MI355X (gfx950).

The compute lives in libkbl.so (hand-written HIP behind the C-ABI of
include/kbl.h); this package only marshals torch tensors into those calls.
Importing it does not load the library; the first call does, and fails
loudly if it has not been built.
"""

from ._lib import (  # noqa: F401
    RS_BAD_INPUT, GRID_GLOBAL, GRID_STENCIL, PREC_FP64, PREC_MIXED_BF16, PREC_MIXED_FP16, PREC_MIXED_FP32,
    ST_INADMISSIBLE, ST_RHO_FLOOR, ST_EPS_RULE, ST_LIMITED, ST_PSTEP, ST_PMEAN_FLOOR,
    ST_MEAN_OUTSIDE, ST_BAD_BOUNDS, ST_BAD_STENCIL, ST_TOO_LARGE, ST_ASYMMETRIC, KblError,
    LIB_PATH,
)
from .fr1d import FR1D  # noqa: F401
from .ops import (  # noqa: F401
    KineticBoundsLimit, autotune_bounds, bounds_and_limit, bounds_limit_backward,
    compute_bounds, compute_bounds_nodes, limit, make_params, make_vgrid, riemann_states,
    status_summary,
)

__all__ = ["compute_bounds", "compute_bounds_nodes", "limit", "riemann_states", "autotune_bounds", "bounds_limit_backward", "bounds_and_limit",
           "KineticBoundsLimit", "status_summary", "make_params", "make_vgrid", "KblError", "FR1D"]
