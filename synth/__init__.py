"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package only *places* inputs: surface nodes of analytic parametrised
surfaces (with the exact parametrisation derivatives), random densities and
incident-wave parameters.  It holds none of the boundary-integral method's
arithmetic (no quadrature weights, no kernels, no interpolation): those live,
independently, in the oracle and in the HIP library.
"""
from .geometry import (Surface, open_cheb_nodes, cube_sphere, ellipsoid,
                       rounded_box, fibonacci_sphere)
from .random import (complex_normal, plane_wave_batch, ellipsoid_batch)

__all__ = ["Surface", "open_cheb_nodes", "cube_sphere", "ellipsoid",
           "rounded_box", "fibonacci_sphere", "complex_normal",
           "plane_wave_batch", "ellipsoid_batch"]
