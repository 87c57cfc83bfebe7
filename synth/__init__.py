"""Seeded synthetic inputs for the filtered time-domain Krylov eigensolver.

This package builds the *inputs* of the method and nothing else: sparse
stiffness matrices ``S`` and lumped (diagonal) mass vectors ``m`` of P1 finite
element discretisations of the Laplacian, start blocks drawn from seeded
normal generators, and the workload recipes that fix mesh, interval and seed.
It holds none of the method's arithmetic (no weights, no time stepping, no
Gram-Schmidt, no Rayleigh-Ritz); both the GPU path and the CPU oracle consume
what it produces.

The discrete problem is the Galerkin pencil ``S v = omega^2 M v`` of Section 2
(definition of ``S`` and ``M``, with ``M`` made diagonal by mass lumping as in
Remark 2.1).
"""

from .grids import (  # noqa: F401
    assemble_p1,
    structured_mesh,
    grid_problem,
    grid_problem_fem,
    prune,
    restrict,
)
from .workloads import (  # noqa: F401
    Problem,
    start_block,
    power_start,
    workload,
    WORKLOADS,
    grid_spectrum,
    distinct_target,
)
