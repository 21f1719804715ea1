"""MI355X (gfx950) implementation of the COSMOS evolution hot path.

The 3+1 Einstein equations in a BSSN (chi) form coupled to a radiation fluid
(P = w rho; centred or Kurganov-Tadmor fluxes) and optionally a massless scalar
field, on a periodic Cartesian grid, in FP64 HIP kernels behind the C ABI of
include/cosmos.h. This package is the thin Python side: ctypes marshalling
(``_lib``) and small drivers that own device buffers (``solver``, ``batch``,
``adjoint``, ``threshold``, ``autotune``).
"""
from . import _lib
from ._lib import (COSMOS_EINVAL, COSMOS_EHIP, COSMOS_OK, NFIELDS, CosmosError, last_error,  # noqa: F401
                   make_grid, make_init, make_params, npts)

# every C-ABI binding (the cosmos_* functions of _lib, one per exported entry point)
for _name in dir(_lib):
    if _name.startswith("cosmos_") and callable(getattr(_lib, _name)):
        globals()[_name] = getattr(_lib, _name)
del _name
from .solver import Solver  # noqa: F401
from .fmr import RefinedRun  # noqa: F401
