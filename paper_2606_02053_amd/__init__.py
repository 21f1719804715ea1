"""MI355X (gfx950) implementation of the COSMOS evolution hot path.

The 3+1 Einstein equations in a BSSN (chi) form coupled to a radiation fluid
(P = w rho; centred or Kurganov-Tadmor fluxes) and optionally a massless scalar
field, on a periodic Cartesian grid, in FP64 HIP kernels behind the C ABI of
include/cosmos.h. This package is the thin Python side: ctypes marshalling
(``_lib``) and small drivers that own device buffers (``solver``, ``batch``,
``adjoint``, ``threshold``, ``autotune``).
"""
from ._lib import (COSMOS_EINVAL, COSMOS_EHIP, COSMOS_OK, NFIELDS, CosmosError, cosmos_abi_version,  # noqa: F401
                   cosmos_adjoint_step, cosmos_adjoint_step_stages, cosmos_adjoint_workspace_bytes, cosmos_rhs_vjp,
                   cosmos_constraints, cosmos_init_fields, cosmos_init_tangent, cosmos_kt_divergence, cosmos_rhs,
                   cosmos_rk4_step, cosmos_rk4_step_stages, cosmos_scalar_workspace_bytes, cosmos_init_fields_scalar,
                   cosmos_rhs_scalar, cosmos_rk4_step_scalar, cosmos_constraints_scalar, cosmos_status, cosmos_status_reset, cosmos_workspace_bytes, last_error,
                   make_grid, make_init, make_params, npts)
from .solver import Solver  # noqa: F401
