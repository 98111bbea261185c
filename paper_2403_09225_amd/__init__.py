"""MI355X-native unbinned partial-wave-analysis likelihood (arXiv:2403.09225).

The HIP library libpwa.so (C ABI in include/pwa.h) evaluates the NLL of
eq. (3), its gradient (eq. (6)) and Hessian-vector product (eq. (7)) and runs
Newton-CG fits; this package is its thin Python binding.
"""

from .api import Likelihood, combine  # noqa: F401
from .autograd import NLLFunction, GradFunction, nll  # noqa: F401
