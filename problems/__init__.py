"""Seeded synthetic inputs for the domain-decomposed ILU0 path.

This package only builds inputs (matrices, right-hand sides, probe vectors).
It contains none of the method's arithmetic: no partitioning, reordering,
factorisation or solve.  Both the CPU oracle and the GPU library consume the
same arrays, so a parity test compares the two on identical data.
"""

from .generators import (  # noqa: F401
    Problem,
    stencil_pattern,
    grid_graph,
    unstructured_problem,
    laplacian_scalar,
    laplacian_blocks,
    random_blocks,
    lognormal_field,
    lognormal_problem,
    training_problem,
    probe_vectors,
    lic_init_params,
    training_order,
    WORKLOADS,
    make_workload,
)
