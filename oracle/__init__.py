"""Plain FP64 CPU oracle for the unbinned partial-wave-analysis likelihood.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or execute anything here; only the test
suite, the package smoke check and the benchmark's CPU-baseline leg use it.
It shares no code with the HIP path.
"""

from .pwa_oracle import (  # noqa: F401
    Dual, DomainError, new_tag, primal, kallen, kinematics, barrier, legendre,
    breakup_sq, amplitude, amplitudes, intensity, nll, partials, combine, grad,
    hvp, hessian, grad_scale, hvp_scale, gram, round_to, fixed_slices, sliced_product,
    nll_batched, newton_cg_fit,
    fraction_matrix, fit_fractions, bfgs_fit, phase_space_factor, flatte_factor, lineshape_of,
    parent_spin, n_helicities, daughter_momenta, angular_factors, helicity_amplitudes,
)
from . import pwa_oracle  # noqa: F401
