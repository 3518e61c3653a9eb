"""MI355X (gfx950) time-level solver for the time-space fractional
convection-diffusion equation of Gu, Huang, Ji, Carpentieri and Alikhanov
(arXiv:1603.00279): the implicit difference scheme's per-level right-hand side
with the L2-1sigma history sum, and the Strang-preconditioned CGS solve of the
nonsymmetric Toeplitz system, in hand-written HIP kernels behind a C ABI
(include/tsfcde.h).
"""
from ._native import (  # noqa: F401
    TSFCDE_OK, TSFCDE_EINVAL, TSFCDE_ENOMEM, TSFCDE_EDEVICE, TSFCDE_ENOCONV, TSFCDE_EBREAKDOWN,
    TSFCDE_ENONFINITE, TSFCDE_EDONE, TSFCDE_EUNSUPPORTED, TSFCDE_EACCEPT, TSFCDE_FP64, TSFCDE_FP32_REFINED,
    TSFCDE_FP32_REFINED_FELL_BACK, TSFCDE_WS_ZERO, TSFCDE_WS_PREV, TSFCDE_WS_EXTRAP, TSFCDE_WS_NET,
    TSFCDE_FLAG_TRUE_RESIDUAL, TSFCDE_FLAG_VERIFY, TSFCDE_FLAG_FORCE_FP32, TSFCDE_FLAG_NO_FOLD,
    TSFCDE_FLAG_STRICT_RESIDUAL, TSFCDE_FLAG_CONSTANT_GSF, TSFCDE_FLAG_GRAPHS, TSFCDE_FLAG_NO_TUNE, TSFCDE_METHOD_PCGS, TSFCDE_METHOD_GSF,
    TSFCDE_METHOD_PBICGSTAB, TSFCDE_KRYLOV_CGS, TSFCDE_KRYLOV_BICGSTAB, TSFCDE_PREC_STRANG, TSFCDE_PREC_TCHAN,
    TSFCDE_OP_A,
    TSFCDE_OP_B, TSFCDE_OP_PINV, TSFCDE_SPEC_EMBED, TSFCDE_SPEC_STRANG, TsfcdeError, lib, header_symbols,
)
from .solver import BatchSolver, TimeLevelSolver  # noqa: F401
from .solver2d import TimeLevelSolver2D  # noqa: F401
from .solver3d import TimeLevelSolver3D  # noqa: F401
from .warmnet import WarmStartNet  # noqa: F401
