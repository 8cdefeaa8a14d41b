"""Seeded synthetic inputs shared by the HIP path, the oracle, the tests and the benchmark.

This package holds only input generation: surface meshes, sample points and the
closed-form boundary data of the test problems.  It contains none of the boundary
element method's arithmetic (no quadrature, no temporal antiderivatives, no
assembly), so that the oracle and the HIP path can both consume its outputs while
sharing no code with each other.
"""
from .meshes import (cube, cube4, icosphere, tetrahedron, octahedron, cubed_sphere_ellipsoid,
                     two_separated_triangles, mesh_summary)
from .points import ball_points, box_points, space_time_points
from .data import (heat_kernel_solution, heat_kernel_flux, exp_solution, nodal_samples,
                   ExactSolution)

__all__ = [
    "cube", "cube4", "icosphere", "tetrahedron", "octahedron", "cubed_sphere_ellipsoid",
    "two_separated_triangles", "mesh_summary", "ball_points", "box_points",
    "space_time_points", "heat_kernel_solution", "heat_kernel_flux", "exp_solution",
    "nodal_samples", "ExactSolution",
]
