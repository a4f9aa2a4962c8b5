"""MI355X-native FWIME hot path: HIP kernels for gfx950 behind a C ABI.

Operators (Section 2 of Barnier et al., arXiv 2206.02362): nonlinear
acoustic modeling, extended (horizontal subsurface-offset) Born modeling and
its adjoint, and the FWIME objective with its gradients.  See include/fwime.h.
"""
from ._abi import (  # noqa: F401
    EXPORTED,
    FWIME_EHIP,
    FWIME_EINVAL,
    FWIME_ENOMEM,
    FWIME_ENONFINITE,
    FWIME_OK,
    FWIME_OP_BORN_ADJ,
    FWIME_OP_BORN_FWD,
    FWIME_OP_GRADIENT,
    FWIME_OP_MODEL,
    LIB_PATH,
    Context,
    Engine,
    FwimeError,
    Geometry,
    Grid,
    Tape,
    footprint,
    load,
)
from .autograd import FwimeOp, predicted_data  # noqa: F401,E402
