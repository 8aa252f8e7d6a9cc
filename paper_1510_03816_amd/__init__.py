"""MI355X-native geodesic landmark shooting with the N-particle Euler-Poincare system.

The computation lives in the HIP library liblm.so (C ABI in include/liblm.h); this package
is its Python binding.  Importing it loads the library and fails loudly if it is missing:
there is no CPU path.
"""

from ._lib import (  # noqa: F401
    CONON, GAUSS, F64, F32, SOLVE_AUTO, SOLVE_CG, SOLVE_DENSE, EXPORTS, LmError, STATUS_NAMES,
    LM_OK, LM_EINVAL, LM_ENOMEM, LM_EHIP, LM_ENOTCONV, LM_EDIVERGED, LM_ESINGULAR, LM_EUNSUPPORTED,
    lm_params, lm_match_opts, lm_match_info, lm_step_info, make_params, last_error, load,
    lm_rhs, lm_shoot, lm_shoot_noalloc, lm_hamiltonian, lm_ksolve, lm_feedback_match, lm_feedback_step, lm_velocity, lm_flow_points,
    lm_version, lm_rhs_vjp, lm_shoot_adjoint, lm_energy_grad, lm_lbfgs_match, lm_lbfgs_opts, lm_lbfgs_info,
    lm_batch_tuning, lm_batch_default_tuning, lm_batch_autotune, lm_rhs_batched, lm_shoot_batched,
    lm_feedback_match_batched, lm_plan_info, lm_pair_plan,
)

load()

from . import autograd  # noqa: E402,F401
