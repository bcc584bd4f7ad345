"""Seeded synthetic inputs for the radiative-transfer step.

This module builds the per-cell fields (density, temperature, velocity,
opacities), the initial intensities and the run parameters of the test and
benchmark workloads.  It holds none of the method's arithmetic: it only draws
random numbers and evaluates the initial/boundary conditions that define each
workload.  Both the CPU oracle and the GPU library consume exactly the arrays
produced here.

Conventions (shared by both consumers):
  * a grid is ``(nx, ny, nz)``; a cell index is ``x + nx*(y + ny*z)`` (x
    fastest), so per-cell arrays are flat ``float64`` arrays of length
    ``nx*ny*nz``;
  * velocity is a ``(3, ncell)`` array (component-major);
  * intensities are ``(nang, ncell)`` arrays (angle-major);
  * boundary codes: 0 periodic, 1 fixed ghost intensities (per-face, per-angle
    table), 2 copy of the last active cell for every angle, 3 vacuum (outgoing
    angles copied, incoming set to zero).
"""
from .configs import (  # noqa: F401
    BC_PERIODIC, BC_FIXED, BC_COPY, BC_VACUUM,
    Workload, config1, config2, config3, config4_requests, config5, request_workload,
    small_case, equilibrium_intensity, moment_intensity, lognormal,
)
from .atmosphere import atmosphere  # noqa: F401
from .beams import (  # noqa: F401
    crossing_beams, direction_at, plane_directions, shadow2d, shadow_density,
)
