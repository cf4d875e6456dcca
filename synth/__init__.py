"""Seeded synthetic inputs shared by the oracle checks, the GPU tests and the bench.

This package only *makes inputs*: meshes, element stencils (CSR), nodal fields
in conserved variables, element quadrature weights and limiter targets.  It
holds none of the bounds/limiter arithmetic, so the oracle and the HIP path
stay independent of each other while consuming byte-identical arrays.
"""

from .workloads import (  # noqa: F401
    Workload,
    GridSpec,
    make_workload,
    make_line_workload,
    make_quad_workload,
    make_tri_workload,
    make_quad_fr_workload,
    make_hex_workload,
    NodeWorkload,
    sample_elements,
    WORKLOADS,
)
