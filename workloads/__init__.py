"""Seeded synthetic finite-element workloads.

This package only *produces inputs*: meshes, assembled CSR matrices and the
random vectors that go with them.  It holds none of the arithmetic of the
sparse matrix-vector product or of the conjugate-gradient solver, so both the
CPU oracle and the HIP library can be driven from it without sharing code.

Every random draw comes from ``numpy.random.default_rng([cfg, purpose, idx])``
(PCG64) with ``purpose`` one of the constants in :mod:`workloads.seeds`.
"""
from .seeds import rng, JITTER, PERM, XVEC, BVEC, SIZES, ARRIVALS  # noqa: F401
from .meshes import (  # noqa: F401
    CSR,
    poisson_2d_p1,
    laplace_1d_p1,
    tet_p1,
    tet_p2,
    hex_q1,
    graded_2d_p1,
    structured_grid,
)
from .configs import (  # noqa: F401
    config0_poisson2d,
    config1_elasticity3d,
    sweep_matrix,
    SWEEP,
    random_vector,
)
