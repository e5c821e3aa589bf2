"""Seeded synthetic particle sets shared by the oracle, the tests and the benchmark.

This package draws positions and masses only. It holds none of the method's arithmetic, so the
CPU oracle and the HIP path can both take their inputs from it without sharing any code.
"""
from .generators import (  # noqa: F401
    Particles,
    uniform_cube,
    plummer_sphere,
    clustered_spheres,
    gridlet_node_lattice,
    point_source_with_tracers,
    random_subset,
    workload,
    WORKLOADS,
    batch_requests,
    serve_requests,
    request_particles,
)
