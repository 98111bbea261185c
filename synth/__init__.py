"""Seeded synthetic inputs shared by the CPU oracle and the HIP path.

This package holds workload definitions (decay masses, resonance tables,
parameter draws) and event generators (phase space, structured data-like
samples, generic accept-reject). It contains none of the likelihood method's
arithmetic: amplitudes, intensities and likelihoods live in the oracle and in
the HIP library, each written separately. Where a generator needs an
intensity (accept-reject), the caller passes it in.
"""

from .workloads import (  # noqa: F401
    PARENT_MASS, DAUGHTER_MASSES, R_BARRIER, CHANNEL_PAIRS, FLATTE_MASSES, FLATTE_RATIO, FLATTE_F0,
    Workload, workload, rng_for, draw_theta, resonance_layout,
)
from .events import (  # noqa: F401
    pair_range, s13_range, bounding_box, uniform_phase_space,
    mirror_symmetric, midpoint_line_s12, midpoint_grid, resonant_like, accept_reject,
    uniform_orientation,
)
