"""Seeded synthetic workloads shared by the oracle, the tests and the benchmark.

This package only draws inputs: marker positions, body centres, prescribed
rigid velocities and grid parameters.  It holds none of the method's
arithmetic (no kernels, operators, velocities at markers or solves), so the
oracle and the GPU path can both consume it without sharing any code of the
method itself.
"""
from .workloads import (  # noqa: F401
    Problem,
    fibonacci_sphere,
    disk_ring,
    sample_centres,
    config0_disk2d,
    config1_sphere3d,
    config2_spheres_ns,
    config4_spheres256,
    small_problem,
    serving_trace,
    icosphere_unit,
    icosphere_spacing,
    shell_problem,
    sedimentation_problem,
    concentric_shells,
    single_shell,
    slit_problem,
    slit_shell,
    box_problem,
    box_shell,
    array_shell,
)
