"""MI355X-native tau-preconditioned GMRES for the penalized 2-D Riesz
space-fractional diffusion equation (Huang & Sun, arXiv 2102.11576).

The computation lives in librsfde.so (HIP kernels for gfx950 behind the C ABI
of include/rsfde.h); this package only marshals arguments.  Importing it
raises ImportError when the library has not been built.
"""

from . import _lib  # noqa: F401  (fails loudly without the HIP library)
from ._lib import (  # noqa: F401
    RsfdeError, make_opts, rsfde_setup, rsfde_set_coeffs, rsfde_matvec, rsfde_precond_apply,
    rsfde_step, rsfde_solve, rsfde_adjoint_step, rsfde_destroy, strerror,
    RSFDE_F_NONE, RSFDE_F_LOGISTIC, RSFDE_F_SIN, RSFDE_F_CUBIC,
)
from .solver import RsfdePlan, RsfdeBatch, StepStats, march_ensemble  # noqa: F401
