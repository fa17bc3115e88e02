"""Seeded synthetic inputs for the sketch-preconditioned least-squares path.

This package only *builds inputs*: random-feature-method (RFM) collocation
systems for the Poisson and Helmholtz problems, test points, exact solutions and a few
structured test matrices.  It contains none of the solver's arithmetic (no
sketch, no QR, no LSQR); both the CPU oracle and the GPU path consume what it
produces.
"""

from .poisson import (  # noqa: F401
    RFMSystem,
    CONFIGS,
    build_config,
    poisson_system,
    sample_points,
    exact_solution,
    feature_eval,
)
from .matrices import (  # noqa: F401
    dense_with_condition,
    random_csr,
    csr_from_dense,
    dense_from_csr,
)
