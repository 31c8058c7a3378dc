"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only draws numbers and states workload shapes.  It holds none of
the butterfly method's arithmetic: no phase evaluation, no interpolation, no
factor construction.  Every generator takes an explicit seed and uses NumPy's
PCG64 (``numpy.random.default_rng``), so the oracle and the GPU path see the
same inputs bit for bit.
"""

from .inputs import (  # noqa: F401
    gaussian_vectors,
    sample_rows,
    amplitude_factors,
    orthogonal_mix,
    lowrank_phase,
)
from .configs import (  # noqa: F401
    CONFIGS,
    PHASE_PARAMS,
    Workload,
    SERVING_SHAPES,
    serving_requests,
)
